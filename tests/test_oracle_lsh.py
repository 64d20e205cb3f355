"""Pins for the LSH candidate oracle: brute force over all pairs, identical and disjoint
shingle sets, the banding S-curve 1 - (1 - J^r)^b, repertoire separation."""
import numpy as np
import pytest

import synth
from oracle import lsh
from oracle import minhash as mh


def _sig(rep, M=64):
    return mh.signatures(rep.seqs, rep.lens, M, synth.HASH_SEED)


def test_dict_grouping_equals_bruteforce():
    r = synth.tiny(n_families=60, fam_size=8, seed=3)
    sig = _sig(r)
    a = lsh.candidates(sig, 16, 4)
    b = lsh.candidates_bruteforce(sig, 16, 4)
    c = lsh.candidates_grouped(sig, 16, 4)
    assert a.shape[0] > 50
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_small5k_bruteforce_on_first_thousand():
    r = synth.small5k()
    sig = _sig(r)[:1000]
    assert np.array_equal(lsh.candidates(sig, 16, 4), lsh.candidates_bruteforce(sig, 16, 4))


def test_canonical_form():
    r = synth.tiny(seed=4)
    p = lsh.candidates(_sig(r), 16, 4)
    assert (p[:, 0] < p[:, 1]).all()
    key = p[:, 0] * r.n + p[:, 1]
    assert (np.diff(key) > 0).all()


def test_identical_and_disjoint_sets():
    seqs, lens = synth.encode(["ACDACDACD", "ACDACD", "WWWWWWWW", "ACDEF"], stride=16)
    sig = mh.signatures(seqs, lens, 64, synth.HASH_SEED)
    p = {tuple(x) for x in lsh.candidates(sig, 16, 4).tolist()}
    assert (0, 1) in p                      # equal shingle sets: every band equal
    assert (0, 2) not in p and (1, 2) not in p and (2, 3) not in p   # disjoint sets


def test_row_helper_matches():
    r = synth.tiny(seed=5)
    sig = _sig(r)
    full = lsh.candidates(sig, 16, 4)
    for i in range(0, r.n, 7):
        row = full[full[:, 0] == i, 1]
        assert np.array_equal(row, lsh.candidates_of_row(sig, i, 16, 4))


def test_repertoires_do_not_mix():
    r = synth.tiny(n_families=30, fam_size=6, seed=6)
    sig = _sig(r)
    sig2 = np.concatenate([sig, sig])           # the same repertoire twice
    offs = [0, r.n, 2 * r.n]
    p = lsh.candidates(sig2, 16, 4, rep_offsets=offs)
    assert (lsh.rep_ids(2 * r.n, offs)[p[:, 0]] == lsh.rep_ids(2 * r.n, offs)[p[:, 1]]).all()
    one = lsh.candidates(sig, 16, 4)
    assert p.shape[0] == 2 * one.shape[0]
    assert np.array_equal(lsh.candidates_bruteforce(sig2, 16, 4, offs), p)


def test_b_times_r_must_fit():
    with pytest.raises(ValueError):
        lsh.candidates(np.zeros((3, 8), np.uint64), 3, 4)


@pytest.mark.slow
def test_s_curve():
    """Empirical P(candidate | J) against 1 - (1 - J^r)^b for 32 x 4 banding."""
    rng = np.random.default_rng(21)
    M, b, r = 128, 32, 4
    T = mh.hash_tables(synth.HASH_SEED, M)
    bins = {}
    for _ in range(4000):
        L = int(rng.integers(10, 21))
        a = list(rng.integers(0, 20, L))
        c = list(a)
        for p in rng.choice(L, int(rng.integers(1, 7)), replace=False):
            c[p] = int((c[p] + rng.integers(1, 20)) % 20)
        J = mh.jaccard(a, c)
        sa, sc = mh.signature(a, T), mh.signature(c, T)
        hit = bool((sa[: b * r].reshape(b, r) == sc[: b * r].reshape(b, r)).all(1).any())
        k = int(J * 10)
        bins.setdefault(k, []).append((J, hit))
    for k, vals in bins.items():
        if len(vals) < 150:
            continue
        Js = np.array([v[0] for v in vals])
        hits = np.array([v[1] for v in vals], dtype=float)
        expect = np.mean([lsh.collision_probability(J, b, r) for J in Js])
        se = np.sqrt(max(expect * (1 - expect), 1e-4) / len(vals))
        assert abs(hits.mean() - expect) < 5 * se + 0.02, (k, hits.mean(), expect)
