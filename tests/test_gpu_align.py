"""GPU Smith-Waterman scores against the C oracle: bit-exact int32."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, oracle_candidates, oracle_scores, say, sw_oracle, workload
from oracle import sw as osw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    return synth.load_blosum62()


def _gpu(seqs, lens, pairs, S, go=10, ge=1, nows=False):
    fn = sq.align_nows if nows else sq.align
    out = fn(dev(seqs), dev(lens), dev(np.asarray(pairs, np.int32)), dev(S), go, ge)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_all_pairs_first_thousand(S):
    r = workload("small5k")
    iu, ju = np.triu_indices(1000, 1)
    pairs = np.stack([iu, ju], 1).astype(np.int32)
    say("align small5k all pairs 1000")
    got = _gpu(r.seqs, r.lens, pairs, S)
    assert np.array_equal(got, sw_oracle(r.seqs, r.lens, pairs, S))


@pytest.mark.parametrize("go,ge", [(10, 1), (1, 1), (5, 0), (0, 0), (1000, 1000), (11, 2)])
def test_gap_costs_and_lengths(S, go, ge):
    rng = np.random.default_rng(go * 7 + ge)
    n, stride = 400, 64
    lens = rng.integers(1, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    # related pairs too: copies with a few edits share long diagonals and gaps
    seqs[1::2, :] = seqs[0::2, :]
    lens[1::2] = lens[0::2]
    for i in range(1, n, 2):
        L = lens[i]
        for p in rng.choice(L, min(L, 3), replace=False):
            seqs[i, p] = rng.integers(0, 20)
    pairs = np.stack([rng.integers(0, n, 3000), rng.integers(0, n, 3000)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], 1)]).astype(np.int32)
    say(f"align random lengths go={go} ge={ge}")
    got = _gpu(seqs, lens, pairs, S, go, ge)
    assert np.array_equal(got, sw_oracle(seqs, lens, pairs, S, go, ge))


def _random_rows(rng, n, stride, lmin=1):
    lens = rng.integers(lmin, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    seqs[1::2, :] = seqs[0::2, :]  # related pairs: copies with a few edits
    lens[1::2] = lens[0::2]
    for i in range(1, n, 2):
        for p in rng.choice(lens[i], min(lens[i], 3), replace=False):
            seqs[i, p] = rng.integers(0, 20)
    return seqs, lens


@pytest.mark.parametrize("go,ge", [(10, 1), (1, 1), (5, 0), (0, 0), (1000, 1000), (11, 2)])
def test_packed_path_gap_costs_and_lengths(S, go, ge):
    """Rows of 32 bytes (the packed half-precision path: two pairs per lane), lengths 1-32 in
    every bucket, odd pair counts (a lane with one pair), all gap settings, against the oracle."""
    rng = np.random.default_rng(100 + go * 7 + ge)
    n, stride = 500, 32
    seqs, lens = _random_rows(rng, n, stride)
    pairs = np.stack([rng.integers(0, n, 4001), rng.integers(0, n, 4001)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], 1)]).astype(np.int32)
    say(f"align packed path go={go} ge={ge}")
    got = _gpu(seqs, lens, pairs, S, go, ge)
    assert np.array_equal(got, sw_oracle(seqs, lens, pairs, S, go, ge))


@pytest.mark.parametrize("top", [64, 65, 127])
def test_packed_path_score_bound(top):
    """A symmetric matrix whose largest score times 32 rows is exactly the packed path's
    bound (64: 2048, every value still exact in half precision) or above it (65, 127: the
    block falls back to int32), on long self-similar pairs that reach the largest scores."""
    rng = np.random.default_rng(top)
    A = rng.integers(-20, 20, (20, 20))
    A = np.triu(A) + np.triu(A, 1).T
    np.fill_diagonal(A, top)
    A = A.astype(np.int8)
    n, stride = 300, 32
    seqs, lens = _random_rows(rng, n, stride, lmin=20)
    pairs = np.stack([rng.integers(0, n, 3000), rng.integers(0, n, 3000)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, np.stack([np.arange(n), np.arange(n)], 1)]).astype(np.int32)
    say(f"align packed path bound top={top}")
    got = _gpu(seqs, lens, pairs, A, 10, 1)
    ref = sw_oracle(seqs, lens, pairs, A, 10, 1)
    assert np.array_equal(got, ref)
    assert ref.max() >= 20 * top  # the self pairs reach the large scores


def test_self_pairs_and_self_scores(S):
    r = synth.tiny(seed=3, Lmin=3, Lmax=32)
    pairs = np.stack([np.arange(r.n), np.arange(r.n)], 1).astype(np.int32)
    say("align self pairs")
    got = _gpu(r.seqs, r.lens, pairs, S)
    diag = osw.self_scores(r.seqs, r.lens, S)
    assert np.array_equal(got, diag)
    ss = sq.self_scores(dev(r.seqs), dev(r.lens), dev(S)).cpu().numpy()
    assert np.array_equal(ss, diag)


def test_without_workspace_entry_point(S):
    r = workload("small5k")
    pairs = synth.random_pairs(r.n, 5000, 8, family=r.family)
    say("align no-workspace entry point")
    a = _gpu(r.seqs, r.lens, pairs, S, nows=True)
    b = _gpu(r.seqs, r.lens, pairs, S)
    assert np.array_equal(a, b)
    assert np.array_equal(a, sw_oracle(r.seqs, r.lens, pairs, S))


def test_empty_and_single(S):
    r = synth.tiny()
    say("align empty / single")
    assert _gpu(r.seqs, r.lens, np.zeros((0, 2), np.int32), S).shape == (0,)
    one = np.array([[0, 1]], np.int32)
    assert np.array_equal(_gpu(r.seqs, r.lens, one, S), sw_oracle(r.seqs, r.lens, one, S))


def test_single_residue_sequences(S):
    seqs = np.full((20, 4), synth.PAD, np.uint8)
    seqs[:, 0] = np.arange(20)
    lens = np.ones(20, np.int32)
    iu, ju = np.meshgrid(np.arange(20), np.arange(20), indexing="ij")
    pairs = np.stack([iu.ravel(), ju.ravel()], 1).astype(np.int32)
    say("align single residues")
    got = _gpu(seqs, lens, pairs, S)
    assert np.array_equal(got, np.maximum(0, S[iu.ravel(), ju.ravel()]).astype(np.int32))


def test_zipf100k_pairs_sampled(S):
    r = workload("zipf100k")
    pairs = synth.random_pairs(r.n, 400_000, 9, family=r.family, same_frac=0.8)
    say("align zipf100k 400k pairs")
    got = _gpu(r.seqs, r.lens, pairs, S)
    sel = synth.sample_rows(pairs.shape[0], 40_000, 1)
    assert np.array_equal(got[sel], sw_oracle(r.seqs, r.lens, pairs[sel], S))


def test_fine_row_buckets_sampled(S):
    """From 2^24 pairs the alignment takes rows buckets of 4 instead of 8 (less padding, more
    launches): over 2^24 family-heavy pairs of the 100k-sequence repertoire (shorter lengths
    8-25, every bucket), a seeded sample of 200,000 scores against the oracle, and every
    score of the first and last 50,000 sorted positions' worth of pairs equal to the same
    pairs aligned in a call below the threshold."""
    r = workload("zipf100k")
    pairs = synth.random_pairs(r.n, 18_500_000, 11, family=r.family, same_frac=0.7)
    assert pairs.shape[0] >= 1 << 24  # (duplicates drawn are dropped)
    say(f"align fine buckets P={pairs.shape[0]}")
    got = _gpu(r.seqs, r.lens, pairs, S)
    sel = synth.sample_rows(pairs.shape[0], 200_000, 4)
    assert np.array_equal(got[sel], sw_oracle(r.seqs, r.lens, pairs[sel], S))
    head = np.ascontiguousarray(pairs[:2_000_000])
    assert np.array_equal(got[:2_000_000], _gpu(r.seqs, r.lens, head, S))


def test_length_sort_with_long_scan(S):
    """2^26 + 2^20 pairs: the length sort's histogram scan then has more than 1024 chunks of
    4096 counters, so it takes its three-launch form (a single-block scan of the chunk totals
    between the two passes).  Random pairs of the 5,000-sequence workload; a seeded sample of
    100,000 scores against the oracle, and the first 1,000,000 equal to the same pairs aligned
    alone (a scan of few chunks)."""
    r = workload("small5k")
    P = (1 << 26) + (1 << 20)
    assert P * 256 // 4096 // 4096 > 1024  # counters of the one 8-bit pass, in chunks
    rng = np.random.default_rng(2026)
    pairs = rng.integers(0, r.n, (P, 2), dtype=np.int32)
    say(f"align long scan P={P}")
    got = _gpu(r.seqs, r.lens, pairs, S)
    sel = synth.sample_rows(P, 100_000, 6)
    assert np.array_equal(got[sel], sw_oracle(r.seqs, r.lens, pairs[sel], S))
    head = np.ascontiguousarray(pairs[:1_000_000])
    assert np.array_equal(got[:1_000_000], _gpu(r.seqs, r.lens, head, S))


def test_rep1m_pairs_sampled(S):
    """Full-size workload: 4M family-heavy pairs over 1M sequences, sampled check."""
    r = workload("rep1m")
    pairs = synth.random_pairs(r.n, 4_000_000, 10, family=r.family, same_frac=0.6)
    say("align rep1m 4M pairs")
    got = _gpu(r.seqs, r.lens, pairs, S)
    sel = synth.sample_rows(pairs.shape[0], 100_000, 2)
    assert np.array_equal(got[sel], sw_oracle(r.seqs, r.lens, pairs[sel], S))
    assert got.min() >= 0


def test_rep1m_candidates_full(S):
    """Every LSH candidate pair of the 1M-sequence workload (the pairs the benchmark aligns),
    in the order the candidate stage emits them, against the C oracle score by score."""
    r = workload("rep1m")
    pairs = oracle_candidates("rep1m").astype(np.int32)
    say(f"align rep1m candidates P={pairs.shape[0]}")
    got = _gpu(r.seqs, r.lens, pairs, S)
    say("align rep1m candidates: oracle scores")
    assert np.array_equal(got, oracle_scores("rep1m"))


def test_asymmetric_matrix(S):
    """An asymmetric substitution matrix: subst[a][b] scores residue a of the pair's first
    sequence against b of its second, whichever is shorter (the kernel's second pass over
    pairs whose operands it swaps uses the transposed table).  Both orders of every pair, all
    lengths 1-64, against the oracle."""
    rng = np.random.default_rng(77)
    A = np.clip(S.astype(np.int64) + rng.integers(-6, 7, (20, 20)), -30, 30).astype(np.int8)
    assert not (A == A.T).all()
    n, stride = 300, 64
    lens = rng.integers(1, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    pairs = np.stack([rng.integers(0, n, 4000), rng.integers(0, n, 4000)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, pairs[:, ::-1]]).astype(np.int32)
    for go, ge in ((10, 1), (3, 2)):
        say(f"align asymmetric matrix go={go} ge={ge}")
        got = _gpu(seqs, lens, pairs, A, go, ge)
        ref = sw_oracle(seqs, lens, pairs, A, go, ge)
        assert np.array_equal(got, ref)
        assert not np.array_equal(ref[:4000], ref[4000:])   # the orientation matters
        assert np.array_equal(_gpu(seqs, lens, pairs, A, go, ge, nows=True), ref)


def test_asymmetric_edit_costs():
    """The edit-distance channel with an asymmetric cost matrix, both orders of every pair."""
    from oracle import edit as oedit
    rng = np.random.default_rng(78)
    C = rng.integers(0, 5, (20, 20)).astype(np.int8)
    np.fill_diagonal(C, 0)
    n, stride = 200, 64
    lens = rng.integers(1, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    pairs = np.stack([rng.integers(0, n, 3000), rng.integers(0, n, 3000)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, pairs[:, ::-1]]).astype(np.int32)
    say("edit distance asymmetric costs")
    out = sq.edit_distance(dev(seqs), dev(lens), dev(pairs), dev(C), indel=3)
    torch.cuda.synchronize()
    ref = oedit.distances_pairs(seqs, lens, pairs, C, 3)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert not np.array_equal(ref[:3000], ref[3000:])
