"""GPU MinHash signatures against the oracle: bit-exact."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, host_u64, oracle_sig, say, workload
from oracle import minhash as omh

pytestmark = pytest.mark.gpu


def test_small5k_exact():
    r = workload("small5k")
    say("minhash small5k M=64")
    got = host_u64(sq.minhash(dev(r.seqs), dev(r.lens), 64))
    torch.cuda.synchronize()
    assert np.array_equal(got, oracle_sig("small5k"))


@pytest.mark.parametrize("M", [1, 5, 63, 64, 65, 100, 128, 200, 256])
def test_sketch_sizes(M):
    r = synth.tiny(n_families=30, fam_size=5, seed=M, Lmin=3, Lmax=32)
    say(f"minhash tiny M={M}")
    got = host_u64(sq.minhash(dev(r.seqs), dev(r.lens), M, seed=12345))
    torch.cuda.synchronize()
    assert np.array_equal(got, omh.signatures(r.seqs, r.lens, M, 12345))


@pytest.mark.parametrize("stride", [4, 8, 12, 64])
def test_strides(stride):
    rng = np.random.default_rng(stride)
    n = 300
    lens = rng.integers(3, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    say(f"minhash stride={stride}")
    got = host_u64(sq.minhash(dev(seqs), dev(lens), 128))
    torch.cuda.synchronize()
    assert np.array_equal(got, omh.signatures(seqs, lens, 128, synth.HASH_SEED))


def test_empty_batch():
    say("minhash n=0")
    out = sq.minhash(torch.zeros((0, 32), dtype=torch.uint8, device="cuda"),
                     torch.zeros(0, dtype=torch.int32, device="cuda"), 64)
    assert out.shape == (0, 64)


def test_check_seqs_reports():
    r = synth.tiny()
    say("check_seqs")
    assert sq.check_seqs(dev(r.seqs), dev(r.lens)) == 0
    bad = r.seqs.copy()
    bad[3, 1] = 25
    with pytest.raises(sq.SubquadError) as ei:
        sq.check_seqs(dev(bad), dev(r.lens))
    assert ei.value.status == 2
    badl = r.lens.copy()
    badl[0] = 2
    with pytest.raises(sq.SubquadError) as ei:
        sq.check_seqs(dev(r.seqs), dev(badl))
    assert ei.value.status == 3


def test_rep1m_full_exact():
    """Full 1M-sequence workload (the launch configuration the benchmark times)."""
    r = workload("rep1m")
    say("minhash rep1m M=128")
    got = host_u64(sq.minhash(dev(r.seqs), dev(r.lens), 128))
    torch.cuda.synchronize()
    ref = oracle_sig("rep1m")
    assert np.array_equal(got, ref)


def test_profile_only_times_the_named_kernel():
    """Kernel timing limited to one kernel records that kernel's launches and no other."""
    from paper_2602_17330_amd import _lib
    r = synth.tiny(n_families=20, fam_size=5)
    s, l = dev(r.seqs), dev(r.lens)
    say("profile_only minhash3_kernel")
    try:
        _lib.profile_enable(True)
        _lib.profile_only("minhash3_kernel")
        sig = sq.minhash(s, l, 64)
        sq.lsh_candidates(sig, 16, 4)
        torch.cuda.synchronize()
        only = _lib.profile_report()
        _lib.profile_only(None)
        sq.minhash(s, l, 64)
        sq.lsh_candidates(sig, 16, 4)
        torch.cuda.synchronize()
        every = _lib.profile_report()
    finally:
        _lib.profile_only(None)
        _lib.profile_enable(False)
    assert set(only) == {"minhash3_kernel"} and only["minhash3_kernel"][0] == 1
    assert "minhash3_kernel" in every and "lsh_keys_kernel" in every
