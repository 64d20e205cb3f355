"""Pins for the Smith-Waterman (Gotoh) oracle: exhaustive alignment enumeration on tiny
strings, Kadane and longest-common-substring special cases, symmetry and reversal,
single letters, a hand-worked affine-gap case and the self-score identity."""
import numpy as np
import pytest

import synth
from oracle import sw


def _rand(rng, lo, hi):
    return list(rng.integers(0, 20, int(rng.integers(lo, hi + 1))))


def test_bruteforce_tiny(blosum62):
    rng = np.random.default_rng(1)
    for k in range(40):
        a, b = _rand(rng, 1, 5), _rand(rng, 1, 4)
        go, ge = [(10, 1), (3, 1), (2, 2), (1, 1)][k % 4]
        ref = sw.score_bruteforce(a, b, blosum62, go, ge)
        assert sw.score_py(a, b, blosum62, go, ge) == ref
        assert sw.score_c(a, b, blosum62, go, ge) == ref


def test_bruteforce_gappy_matrix():
    """A matrix with strong matches and cheap gaps makes gapped alignments optimal."""
    rng = np.random.default_rng(2)
    S = np.full((20, 20), -3, dtype=np.int8)
    np.fill_diagonal(S, 5)
    for _ in range(25):
        a, b = _rand(rng, 3, 5), _rand(rng, 3, 5)
        a = [x % 4 for x in a]
        b = [x % 4 for x in b]
        ref = sw.score_bruteforce(a, b, S, 2, 1)
        assert sw.score_c(a, b, S, 2, 1) == ref == sw.score_py(a, b, S, 2, 1)


def test_bruteforce_asymmetric_matrix():
    """An asymmetric matrix: subst[a][b] scores a residue of the first string against one of
    the second.  The C loop (pairs entry, both orders) equals the enumeration, and the two
    orders differ where the transposed matrix would give another score."""
    rng = np.random.default_rng(3)
    S = rng.integers(-6, 7, (20, 20)).astype(np.int8)
    S[:4, :4] = [[5, 4, -2, -3], [-4, 6, 3, -1], [2, -5, 4, 1], [-2, 3, -3, 5]]
    differ = 0
    for k in range(30):
        a, b = [x % 4 for x in _rand(rng, 2, 5)], [x % 4 for x in _rand(rng, 2, 4)]
        go, ge = [(3, 1), (2, 1), (10, 1)][k % 3]
        ref_ab = sw.score_bruteforce(a, b, S, go, ge)
        ref_ba = sw.score_bruteforce(b, a, S, go, ge)
        assert ref_ba == sw.score_bruteforce(a, b, S.T, go, ge)
        assert sw.score_c(a, b, S, go, ge) == ref_ab == sw.score_py(a, b, S, go, ge)
        seqs = np.full((2, 8), 0xFF, np.uint8)
        seqs[0, : len(a)], seqs[1, : len(b)] = a, b
        lens = np.array([len(a), len(b)], np.int32)
        got = sw.scores_pairs(seqs, lens, np.array([[0, 1], [1, 0]], np.int32), S, go, ge)
        assert list(got) == [ref_ab, ref_ba]
        differ += ref_ab != ref_ba
    assert differ > 0


def _kadane_diagonals(a, b, S):
    best = 0
    for d in range(-len(a) + 1, len(b)):
        run = 0
        for x in range(len(a)):
            y = x + d
            if 0 <= y < len(b):
                run = max(0, run + int(S[a[x]][b[y]]))
                best = max(best, run)
    return best


def test_no_gaps_is_best_diagonal_segment(blosum62):
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = _rand(rng, 1, 30), _rand(rng, 1, 30)
        assert sw.score_c(a, b, blosum62, 1000, 1000) == _kadane_diagonals(a, b, blosum62)


def _lcsubstr(a, b):
    best = 0
    for i in range(len(a)):
        for j in range(len(b)):
            k = 0
            while i + k < len(a) and j + k < len(b) and a[i + k] == b[j + k]:
                k += 1
            best = max(best, k)
    return best


def test_identity_matrix_is_longest_common_substring():
    S = np.full((20, 20), -100, dtype=np.int8)
    np.fill_diagonal(S, 1)
    rng = np.random.default_rng(4)
    for _ in range(200):
        a, b = _rand(rng, 1, 25), _rand(rng, 1, 25)
        a = [x % 3 for x in a]
        b = [x % 3 for x in b]
        assert sw.score_c(a, b, S, 1000, 1000) == _lcsubstr(a, b)


def test_symmetry_and_reversal(blosum62):
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = _rand(rng, 1, 30), _rand(rng, 1, 30)
        s = sw.score_c(a, b, blosum62)
        assert s == sw.score_c(b, a, blosum62)
        assert s == sw.score_c(a[::-1], b[::-1], blosum62)


def test_single_letters(blosum62):
    for x in range(20):
        for y in range(20):
            assert sw.score_c([x], [y], blosum62) == max(0, int(blosum62[x][y]))


def test_hand_worked_affine_gap(blosum62):
    """a = W^m C^m, b = W^m G^k C^m: the best alignment matches both blocks around one gap
    of length k, scoring m (11 + 9) - (10 + (k - 1) * 1); a gap charged 10 + k * 1 would
    give one less."""
    code = synth.ALPHABET.index
    W, C, G = code("W"), code("C"), code("G")
    for m, k in [(2, 2), (3, 2), (3, 3), (4, 1), (5, 4)]:
        a = [W] * m + [C] * m
        b = [W] * m + [G] * k + [C] * m
        expect = m * (11 + 9) - (10 + (k - 1) * 1)
        assert sw.score_c(a, b, blosum62) == expect
        assert sw.score_py(a, b, blosum62) == expect
    a = [W, W, C, C]
    b = [W, W, G, G, C, C]
    assert sw.score_bruteforce(a, b, blosum62) == 2 * 20 - 11


def test_self_score_is_diagonal_sum(blosum62):
    r = synth.tiny(seed=9, Lmin=3, Lmax=30)
    diag = sw.self_scores(r.seqs, r.lens, blosum62)
    pairs = np.stack([np.arange(r.n), np.arange(r.n)], 1).astype(np.int32)
    assert np.array_equal(sw.scores_pairs(r.seqs, r.lens, pairs, blosum62), diag)
    i = 0
    assert diag[i] == sum(int(blosum62[c][c]) for c in r.seqs[i, : r.lens[i]])


def test_pairs_entry_matches_single(blosum62):
    r = synth.tiny(seed=10)
    pairs = synth.random_pairs(r.n, 300, 1, family=r.family)
    out = sw.scores_pairs(r.seqs, r.lens, pairs, blosum62)
    for p in range(0, pairs.shape[0], 13):
        i, j = pairs[p]
        assert out[p] == sw.score_py(list(r.seqs[i, : r.lens[i]]), list(r.seqs[j, : r.lens[j]]), blosum62)


@pytest.mark.slow
def test_parallel_matches_serial(blosum62):
    r = synth.tiny(seed=12)
    pairs = synth.random_pairs(r.n, 2000, 2)
    a = sw.scores_pairs(r.seqs, r.lens, pairs, blosum62)
    b = sw.scores_pairs_parallel(r.seqs, r.lens, pairs, blosum62, procs=2)
    assert np.array_equal(a, b)
