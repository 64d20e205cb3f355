"""Input generators: encoding, substitution matrix, repertoire structure."""
import numpy as np
import pytest

import synth


def test_encode_roundtrip():
    strings = ["CASSLGQAYEQYF", "ACDEFGHIKLMNPQRSTVWY", "WWW"]
    seqs, lens = synth.encode(strings, stride=32)
    assert seqs.dtype == np.uint8 and seqs.shape == (3, 32)
    assert list(lens) == [13, 20, 3]
    assert [synth.decode(seqs[i], lens[i]) for i in range(3)] == strings
    assert (seqs[0, 13:] == synth.PAD).all()
    assert list(seqs[1, :20]) == list(range(20))


def test_encode_rejects():
    with pytest.raises(ValueError):
        synth.encode(["CASSB"])
    with pytest.raises(ValueError):
        synth.encode(["A" * 40], stride=32)


def test_blosum62_properties(blosum62):
    S = blosum62.astype(int)
    assert S.shape == (20, 20)
    assert (S == S.T).all()
    diag = {c: S[i, i] for i, c in enumerate(synth.ALPHABET)}
    # published diagonal of BLOSUM62
    assert diag == dict(A=4, C=9, D=6, E=5, F=6, G=6, H=8, I=4, K=5, L=4, M=5, N=6, P=7,
                        Q=5, R=5, S=4, T=5, V=4, W=11, Y=7)
    off = S[~np.eye(20, dtype=bool)]
    assert off.min() == -4 and off.max() == 3
    # every off-diagonal entry is below every diagonal entry (self-score identity needs it)
    assert off.max() < S.diagonal().min()
    idx = synth.ALPHABET.index
    assert S[idx("W"), idx("W")] == 11 and S[idx("I"), idx("V")] == 3 and S[idx("F"), idx("Y")] == 3
    assert S[idx("W"), idx("N")] == -4 and S[idx("E"), idx("Q")] == 2 and S[idx("K"), idx("R")] == 2


def test_small5k_structure():
    r = synth.small5k()
    assert r.n == 5000 and r.stride == 32
    assert r.lens.min() >= 8 and r.lens.max() <= 20
    assert np.bincount(r.family).tolist() == [10] * 500
    v = np.ascontiguousarray(r.seqs).view(np.dtype((np.void, 32))).ravel()
    assert np.unique(v).size == r.n
    for i in range(50):
        L = r.lens[i]
        assert (r.seqs[i, :L] < 20).all() and (r.seqs[i, L:] == synth.PAD).all()
    assert abs(r.subgroup.mean() - 0.01) < 1e-9
    r2 = synth.small5k()
    assert (r2.seqs == r.seqs).all() and (r2.vgene == r.vgene).all()


def test_zipf_sizes():
    s = synth.zipf_rank_sizes(100_000, 10_000)
    assert s.sum() == 100_000 and s.min() == 1
    assert (np.diff(s) <= 0).all()
    assert s[0] > 30_000


def test_batch_sizes():
    s = synth.batch_sizes()
    assert s.shape == (64,) and s[0] >= 10_000 and s[-1] <= 2_000_000
    assert 23_000_000 < s.sum() < 25_000_000


def test_embeddings_unit_and_deterministic():
    r = synth.tiny()
    e = synth.embeddings(r.seqs, r.lens, 64)
    assert e.dtype == np.float32 and e.shape == (r.n, 64)
    assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-6)
    assert (synth.embeddings(r.seqs, r.lens, 64) == e).all()


def test_random_pairs_canonical():
    r = synth.tiny()
    p = synth.random_pairs(r.n, 500, 3, family=r.family)
    assert (p[:, 0] < p[:, 1]).all()
    key = p[:, 0].astype(np.int64) * r.n + p[:, 1]
    assert (np.diff(key) > 0).all()
