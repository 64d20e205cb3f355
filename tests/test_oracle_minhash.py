"""Pins for the MinHash oracle: published generator outputs, hash injectivity, identities
of the minimum over a shingle set, and the 1/sqrt(M) sampling error of the Jaccard
estimate (paper, Appendix B, sampling-error bounds)."""
import os

import numpy as np
import pytest

import synth
from oracle import minhash as mh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("seed"):
            head, vals = line.split(":")
            out[int(head.split()[1])] = [int(v, 16) for v in vals.split()]
    return out


def test_splitmix64_published_vectors():
    for seed, vals in _golden().items():
        assert mh.splitmix64(seed, len(vals)) == vals


def test_table_order():
    T = mh.hash_tables(123, 4)
    flat = mh.splitmix64(123, 4 * 60)
    assert int(T[0, 0, 0]) == flat[0] and int(T[0, 0, 19]) == flat[19]
    assert int(T[0, 1, 0]) == flat[20] and int(T[0, 2, 5]) == flat[45]
    assert int(T[1, 0, 0]) == flat[60] and int(T[3, 2, 19]) == flat[239]


@pytest.mark.parametrize("M", [64, 128, 256])
def test_hash_injective_on_all_3mers(M):
    T = mh.hash_tables(synth.HASH_SEED, M)
    a, b, c = np.meshgrid(np.arange(20), np.arange(20), np.arange(20), indexing="ij")
    h = T[:, 0, a.ravel()] ^ T[:, 1, b.ravel()] ^ T[:, 2, c.ravel()]     # [M, 8000]
    hs = np.sort(h, axis=1)
    assert (np.diff(hs, axis=1) != 0).all()


def test_three_residue_sequence_is_its_hash():
    T = mh.hash_tables(synth.HASH_SEED, 64)
    sig = mh.signature([3, 17, 5], T)
    for t in range(64):
        assert int(sig[t]) == int(T[t, 0, 3]) ^ int(T[t, 1, 17]) ^ int(T[t, 2, 5])


def _rand_codes(rng, L):
    return list(rng.integers(0, 20, L))


def test_min_identities():
    rng = np.random.default_rng(5)
    T = mh.hash_tables(synth.HASH_SEED, 64)
    for _ in range(60):
        L = int(rng.integers(4, 25))
        s = _rand_codes(rng, L)
        sig = mh.signature(s, T)
        # the shingle set of s is the union of those of s[:-1] and s[1:]
        assert (sig == np.minimum(mh.signature(s[:-1], T), mh.signature(s[1:], T))).all()
        # a prefix has fewer shingles, so its minimum is not smaller
        assert (mh.signature(s[: L - 1], T) >= sig).all()


def test_equal_shingle_sets_equal_signatures():
    T = mh.hash_tables(synth.HASH_SEED, 128)
    A = [0, 1, 2] * 2        # ACDACD
    B = [0, 1, 2] * 3        # ACDACDACD: same shingle set
    assert mh.shingles(A) == mh.shingles(B)
    assert (mh.signature(A, T) == mh.signature(B, T)).all()
    assert mh.jaccard(A, B) == 1.0


def test_vectorised_matches_set_definition():
    r = synth.tiny(n_families=10, fam_size=5, Lmin=3, Lmax=30)
    T = mh.hash_tables(synth.HASH_SEED, 64)
    sig = mh.signatures(r.seqs, r.lens, 64, synth.HASH_SEED)
    for i in range(r.n):
        assert (sig[i] == mh.signature(r.seqs[i, : r.lens[i]], T)).all()


def test_jaccard_estimate_statistics():
    """z = (J_hat - J) / sqrt(J (1 - J) / M) over many pairs: mean ~0, variance ~1."""
    rng = np.random.default_rng(11)
    M = 128
    T = mh.hash_tables(synth.HASH_SEED, M)
    zs = []
    while len(zs) < 3000:
        L = int(rng.integers(8, 21))
        a = _rand_codes(rng, L)
        b = list(a)
        for p in rng.choice(L, int(rng.integers(1, 5)), replace=False):
            b[p] = int((b[p] + rng.integers(1, 20)) % 20)
        J = mh.jaccard(a, b)
        if not 0.0 < J < 1.0:
            continue
        Jh = mh.jaccard_estimate(mh.signature(a, T), mh.signature(b, T))
        zs.append((Jh - J) / np.sqrt(J * (1 - J) / M))
        assert abs(Jh - J) <= 1.0 / np.sqrt(M) + 4 * np.sqrt(J * (1 - J) / M)
    zs = np.array(zs)
    assert abs(zs.mean()) < 0.08
    assert 0.85 < zs.var() < 1.15


def test_self_estimate_is_one():
    T = mh.hash_tables(synth.HASH_SEED, 64)
    s = [1, 5, 9, 2, 2, 7]
    assert mh.jaccard_estimate(mh.signature(s, T), mh.signature(s, T)) == 1.0


@pytest.mark.parametrize("M", [1, 64, 65, 128, 256])
@pytest.mark.parametrize("stride", [4, 8, 20, 32, 64])
def test_c_loop_matches_set_definition(M, stride):
    """The C loop (minhash_ref.c) against the set-based definition and the vectorised form,
    on edge lengths 3 and stride, repeated 3-mers and ragged rows."""
    rng = np.random.default_rng(1000 + 7 * M + stride)
    n = 24
    lens = rng.integers(3, stride + 1, n).astype(np.int32)
    lens[0], lens[1] = 3, stride
    seqs = np.full((n, stride), 0xFF, dtype=np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    if stride >= 9:
        lens[2] = 9
        seqs[2, :9] = [4, 7, 1] * 3        # one shingle repeated (set of 3 distinct)
    T = mh.hash_tables(synth.HASH_SEED, M)
    c = mh.signatures_c(seqs, lens, M, synth.HASH_SEED)
    v = mh.signatures(seqs, lens, M, synth.HASH_SEED)
    assert c.dtype == np.uint64 and c.shape == (n, M)
    assert np.array_equal(c, v)
    for i in range(n):
        assert np.array_equal(c[i], mh.signature(seqs[i, : lens[i]], T))


def test_c_loop_matches_vectorised_small5k():
    r = synth.small5k()
    M = r.params["M"]
    assert np.array_equal(mh.signatures_c(r.seqs, r.lens, M, synth.HASH_SEED),
                          mh.signatures(r.seqs, r.lens, M, synth.HASH_SEED))
