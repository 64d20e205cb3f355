"""Memory-sized batching (Sec. 3.5, Eq. (batch)) -- host logic."""
import math

from paper_2602_17330_amd.batching import bytes_per_sequence, eq_batch, plan_batches


def test_eq_batch_as_printed():
    # B = min(|S|, max(32, floor(sqrt(M / (c * l)))))
    assert eq_batch(10**6, 288e9, 64.0, 30) == math.floor(math.sqrt(288e9 / (64 * 30)))
    assert eq_batch(100, 288e9, 64.0, 30) == 100
    assert eq_batch(10**6, 1e3, 64.0, 30) == 32


def test_plan_packs_whole_repertoires_in_order():
    sizes = [10, 20, 30, 40, 50]
    plan = plan_batches(sizes, 1.0, 100.0, headroom=1.0)
    assert plan == [[0, 1, 2, 3], [4]]          # 10+20+30+40 = 100 fits exactly
    assert sum(plan, []) == list(range(5))
    # a repertoire larger than the budget still gets a batch of its own
    assert plan_batches([500], 1.0, 100.0) == [[0]]


def test_footprint_grows_with_pairs():
    a = bytes_per_sequence(128, 32, 128, 32, 10)
    b = bytes_per_sequence(128, 32, 128, 32, 40)
    assert b > a > 128 * 8
