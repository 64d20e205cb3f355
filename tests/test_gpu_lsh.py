"""GPU LSH candidates against the oracle: bit-exact pair sets in canonical order."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, oracle_candidates, oracle_sig, pairs_valid, row_candidates_sampled, say, workload
from oracle import lsh as olsh
from oracle import minhash as omh

pytestmark = pytest.mark.gpu


def _gpu(sig_np, b, r, offs=None, cap=None):
    offs_t = dev(np.asarray(offs, np.int64)) if offs is not None else None
    pairs, rows = sq.lsh_candidates(dev(sig_np), b, r, rep_offsets=offs_t, cap=cap)
    torch.cuda.synchronize()
    return pairs.cpu().numpy().astype(np.int64), rows.cpu().numpy()


def _rows_ok(pairs, rows, n):
    return np.array_equal(rows, np.searchsorted(pairs[:, 0], np.arange(n + 1), side="left"))


def test_small5k_exact():
    sig = oracle_sig("small5k")
    say("lsh small5k 16x4")
    got, rows = _gpu(sig, 16, 4)
    ref = olsh.candidates(sig, 16, 4)
    assert got.shape[0] > 1000
    assert np.array_equal(got, ref)
    assert _rows_ok(got, rows, sig.shape[0])


@pytest.mark.parametrize("b,r,M", [(16, 4, 64), (32, 4, 128), (8, 8, 64), (64, 2, 128), (128, 1, 128),
                                   (20, 3, 64), (1, 1, 1)])
def test_band_shapes(b, r, M):
    rep = synth.tiny(n_families=50, fam_size=6, seed=b * 100 + r)
    sig = omh.signatures(rep.seqs, rep.lens, M, synth.HASH_SEED)
    say(f"lsh tiny {b}x{r} M={M}")
    got, rows = _gpu(sig, b, r)
    assert np.array_equal(got, olsh.candidates(sig, b, r))
    assert _rows_ok(got, rows, rep.n)


def test_band_count_limit():
    """b > 256 is refused before any launch (the band must fit the key's spare bits and the
    key kernel's LDS)."""
    sig = np.zeros((10, 300), np.uint64)
    with pytest.raises(sq.SubquadError, match="b <= 256"):
        _gpu(sig, 257, 1)


def test_over_2p20_rows_full_key():
    """n = 2^20 + 12,345 rows: the record sort keeps all 32 mix bits (four passes) and the
    band is compared by division.  Random words from 2^22 values per band, so about 2^17
    chance collisions per band, checked against the oracle."""
    n = (1 << 20) + 12345
    rng = np.random.default_rng(2)
    sig = rng.integers(0, 1 << 22, size=(n, 2), dtype=np.uint64)
    say(f"lsh n={n} 2x1 random words")
    got, rows = _gpu(sig, 2, 1, cap=1 << 20)
    ref = olsh.candidates(sig, 2, 1)
    assert ref.shape[0] > 100_000
    assert np.array_equal(got, ref)
    assert _rows_ok(got, rows, n)


def test_large_identical_bucket():
    """600 copies of one signature: one bucket holding every pair (skewed run)."""
    rep = synth.tiny(n_families=20, fam_size=5, seed=31)
    sig = omh.signatures(rep.seqs, rep.lens, 64, synth.HASH_SEED)
    sig = np.concatenate([sig, np.repeat(sig[:1], 600, axis=0)])
    rng = np.random.default_rng(0)
    sig = sig[rng.permutation(sig.shape[0])]
    say("lsh identical bucket")
    got, rows = _gpu(sig, 16, 4)
    ref = olsh.candidates(sig, 16, 4)
    assert ref.shape[0] >= 601 * 600 // 2
    assert np.array_equal(got, ref)


def test_repertoires_separate():
    reps = [synth.tiny(n_families=20 + 5 * k, fam_size=4, seed=40 + k) for k in range(4)]
    reps.append(reps[0])  # a repeated repertoire: identical signatures, no cross pairs
    batch = synth.concat(reps)
    sig = omh.signatures(batch.seqs, batch.lens, 64, synth.HASH_SEED)
    say("lsh 5 repertoires")
    got, rows = _gpu(sig, 16, 4, offs=batch.rep_offsets)
    ref = olsh.candidates(sig, 16, 4, rep_offsets=batch.rep_offsets)
    assert np.array_equal(got, ref)
    # equal to the per-repertoire results shifted by the offsets
    parts = []
    for k, rp in enumerate(reps):
        o = batch.rep_offsets[k]
        g, _ = _gpu(sig[o:o + rp.n], 16, 4)
        parts.append(g + o)
    assert np.array_equal(got, np.concatenate(parts))


def test_capacity_error_and_retry():
    sig = oracle_sig("small5k")
    ref = olsh.candidates(sig, 16, 4)
    say("lsh capacity error")
    with pytest.raises(sq.SubquadError):
        # a direct call with too small a capacity
        import ctypes
        from paper_2602_17330_amd._lib import lib
        n = sig.shape[0]
        cap = 10
        wsb = lib().subquad_lsh_workspace_bytes(n, 16, cap)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        P = ctypes.c_int64(0)
        s = dev(sig)
        st = lib().subquad_lsh_candidates(s.data_ptr(), n, 64, 16, 4, None, 1, ws.data_ptr(), wsb,
                                          pairs.data_ptr(), None, cap, ctypes.byref(P),
                                          torch.cuda.current_stream().cuda_stream)
        assert st == 4 and P.value == ref.shape[0]
        raise sq.SubquadError(st, "expected")
    got, _ = _gpu(sig, 16, 4, cap=10)   # the binding retries with the reported size
    assert np.array_equal(got, ref)


def test_async_matches_sync():
    import ctypes
    from paper_2602_17330_amd._lib import lib
    sig = oracle_sig("small5k")
    ref = olsh.candidates(sig, 16, 4)
    n = sig.shape[0]
    cap = ref.shape[0] + 100
    say("lsh async")
    wsb = lib().subquad_lsh_workspace_bytes(n, 16, cap)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    rows = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = dev(sig)
    st = lib().subquad_lsh_candidates_async(s.data_ptr(), n, 64, 16, 4, None, 1, ws.data_ptr(), wsb,
                                            pairs.data_ptr(), rows.data_ptr(), cap, cnt.data_ptr(),
                                            status.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    P = int(cnt.item())
    assert status.item() == 0 and P == ref.shape[0]
    assert np.array_equal(pairs[:P].cpu().numpy(), ref)
    # too small a capacity: status flags it, the count is still exact
    st = lib().subquad_lsh_candidates_async(s.data_ptr(), n, 64, 16, 4, None, 1, ws.data_ptr(), wsb,
                                            pairs.data_ptr(), rows.data_ptr(), 50, cnt.data_ptr(),
                                            status.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == 0 and status.item() == 4 and int(cnt.item()) == ref.shape[0]


def test_deterministic():
    sig = oracle_sig("small5k")
    say("lsh determinism")
    a, _ = _gpu(sig, 16, 4)
    b, _ = _gpu(sig, 16, 4)
    assert np.array_equal(a, b)


def test_zipf100k_sampled_rows():
    """Skewed family sizes (head family ~36k): validity of every pair, exact rows sampled."""
    rep = workload("zipf100k")
    sig = oracle_sig("zipf100k")
    say("lsh zipf100k 32x4")
    got, rows = _gpu(sig, 32, 4)
    assert pairs_valid(sig, got, 32, 4)
    key = got[:, 0] * rep.n + got[:, 1]
    assert (np.diff(key) > 0).all()
    head = np.argmax(np.bincount(rep.family))
    sample = np.concatenate([synth.sample_rows(rep.n, 60, 5), np.nonzero(rep.family == head)[0][:20]])
    for i, ref in row_candidates_sampled(sig, sample, 32, 4).items():
        assert np.array_equal(got[rows[i]:rows[i + 1], 1], ref), i


def test_rep1m_full_size():
    """1M sequences, 32x4 (the launch configuration the benchmark times): the whole candidate
    set against the oracle's, pair for pair in canonical order, and the CSR row offsets."""
    rep = workload("rep1m")
    sig = oracle_sig("rep1m")
    say("lsh rep1m 32x4")
    got, rows = _gpu(sig, 32, 4)
    say(f"lsh rep1m: {got.shape[0]} pairs from the GPU; oracle candidate set")
    ref = oracle_candidates("rep1m")
    assert ref.shape[0] > 3_000_000
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    assert _rows_ok(got, rows, rep.n)


def test_edge_cases():
    rep = synth.tiny(n_families=20, fam_size=5, seed=51)
    sig = omh.signatures(rep.seqs, rep.lens, 64, synth.HASH_SEED)
    say("lsh edge cases")
    # a single sequence: no pairs, offsets all zero
    got, rows = _gpu(sig[:1], 16, 4)
    assert got.shape == (0, 2) and np.array_equal(rows, [0, 0])
    # b*r < M: only the first b*r rows take part
    got, _ = _gpu(sig, 5, 3)
    assert np.array_equal(got, olsh.candidates(sig, 5, 3))
    # empty repertoires inside the offsets
    offs = [0, 0, 40, 40, 40, 70, rep.n, rep.n]
    got, _ = _gpu(sig, 16, 4, offs=offs)
    assert np.array_equal(got, olsh.candidates(sig, 16, 4, rep_offsets=offs))


def test_two_thousand_identical():
    """2,000 identical signatures: about 2 million pairs from one bucket in every band."""
    rep = synth.tiny(n_families=10, fam_size=5, seed=52)
    sig = omh.signatures(rep.seqs, rep.lens, 64, synth.HASH_SEED)
    sig = np.concatenate([sig, np.repeat(sig[3:4], 2000, axis=0)])
    say("lsh 2000 identical")
    got, rows = _gpu(sig, 16, 4)
    ref = olsh.candidates_grouped(sig, 16, 4)
    assert ref.shape[0] >= 2001 * 2000 // 2
    assert np.array_equal(got, ref)
