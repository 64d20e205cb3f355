"""Pins for the RMT edge-threshold oracle (Sec. 3.7): the bulk edge against the Wigner
semicircle law, largest eigenvalues against closed forms, and a planted graph whose
threshold is known exactly."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import rmt


def test_bulk_edge_is_the_semicircle_edge():
    """A symmetric matrix with i.i.d. centred entries: its largest eigenvalue approaches
    2 sigma sqrt(n) = 2 sqrt(sum a^2 / n) (finite-size deviation of order n^(-2/3))."""
    rng = np.random.default_rng(0)
    for n, density in ((800, 1.0), (3000, 0.05)):
        X = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
        W = np.triu(X, 1)
        A = sp.csr_matrix(W + W.T)
        ratio = rmt.lambda_max(A) / rmt.bulk_edge(A)
        assert abs(ratio - 1.0) < 0.04, (n, ratio)


def test_lambda_max_closed_forms():
    c = 0.7
    m = 9
    K = sp.csr_matrix(c * (np.ones((m, m)) - np.eye(m)))       # complete graph: c (m - 1)
    assert rmt.lambda_max(K) == pytest.approx(c * (m - 1), rel=1e-12)
    star = np.zeros((m + 1, m + 1))
    star[0, 1:] = star[1:, 0] = c                              # star: c sqrt(m)
    assert rmt.lambda_max(sp.csr_matrix(star)) == pytest.approx(c * np.sqrt(m), rel=1e-12)
    path = np.diag(np.full(m - 1, c), 1)
    path = path + path.T                                      # path: 2 c cos(pi / (m + 1))
    assert rmt.lambda_max(sp.csr_matrix(path)) == pytest.approx(2 * c * np.cos(np.pi / (m + 1)), rel=1e-12)
    assert rmt.lambda_max(sp.csr_matrix((5, 5))) == 0.0


def test_tridiagonal_eigenvalues_of_a_path():
    m = 30
    got = rmt.tridiag_eigvals(np.zeros(m), np.ones(m - 1))
    ref = np.sort(2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1)))
    assert np.allclose(got, ref, atol=1e-12)


def _planted(seed=1, n_match=2000, cliques=50, m=12, w_clique=0.9):
    rng = np.random.default_rng(seed)
    pairs, w = [], []
    node = 0
    for _ in range(n_match):                                  # noise: isolated edges, w < 0.5
        pairs.append((node, node + 1))
        w.append(rng.uniform(0.0, 0.5))
        node += 2
    clique_pairs = []
    for _ in range(cliques):                                  # signal: cliques at exactly w_clique
        for a in range(m):
            for b in range(a + 1, m):
                clique_pairs.append((node + a, node + b))
        node += m
    pairs += clique_pairs
    w += [w_clique] * len(clique_pairs)
    return np.array(pairs, np.int64), np.array(w), node, len(clique_pairs)


def test_planted_cliques_are_exactly_what_is_kept():
    pairs, w, n, nclique = _planted()
    tau, lp, lmax = rmt.threshold(pairs, w, n)
    assert lmax == pytest.approx(0.9 * 11, rel=1e-10)          # a clique's eigenvalue
    assert 0.5 < lp < 0.9 * 11
    assert 0.9 * (1 - 2.0 ** -19) <= tau <= 0.9               # the bisection converges to 0.9 from below
    kept = w >= tau
    assert kept.sum() == nclique and kept[-nclique:].all()


def test_no_structure_keeps_nothing():
    pairs, w, n, nclique = _planted(cliques=0)
    tau, lp, lmax = rmt.threshold(pairs, w, n)
    assert lmax <= lp and tau > w.max()


def test_lambda_max_below_is_monotone_and_bracketed():
    """Perron-Frobenius: adding nonnegative entries never lowers the largest eigenvalue; the
    bisection ends on a bracket [tau, tau + step] across the bulk edge."""
    rng = np.random.default_rng(3)
    n = 400
    P = rng.integers(0, n, (3000, 2))
    w = rng.uniform(0.0, 1.0, 3000) ** 2
    A = rmt.matrix(P, w, n)
    grid = np.linspace(0.0, 1.0, 21)
    lm = [rmt.lambda_max(rmt.below(A, t)) for t in grid]
    assert all(b >= a - 1e-12 for a, b in zip(lm, lm[1:]))
    tau, lp, lmax, trace = rmt.threshold(P, w, n, return_trace=True)
    if lmax > lp:
        step = A.data.max() * 2.0 ** -rmt.ITERS
        assert rmt.lambda_max(rmt.below(A, tau)) <= lp
        assert rmt.lambda_max(rmt.below(A, tau + 1.0001 * step)) > lp


def test_matrix_reading():
    """Negative, NaN and self-pair affinities make no entry; every pair gives both directions."""
    pairs = np.array([[0, 1], [1, 2], [2, 3], [3, 3]])
    w = np.array([0.5, -0.2, np.nan, 0.9])
    A = rmt.matrix(pairs, w, 4).toarray()
    ref = np.zeros((4, 4))
    ref[0, 1] = ref[1, 0] = 0.5
    assert np.array_equal(A, ref)
