"""GPU RMT edge threshold (Sec. 3.7) against the float64 oracle.

Tolerances: lambda_plus is a float64 sum of the same float32 weights (relative 1e-12); a
largest eigenvalue from float32 Lanczos vectors (Rayleigh quotients accurate to about
u |A|) relative 1e-5.  tau* is a sequence of bisection decisions: where every decision of the
oracle's bisection clears the bulk edge by more than the eigenvalue tolerance, tau* must be
the oracle's to the bit; otherwise the GPU's tau* must bracket the edge within that
tolerance (lambda_max of the edges below tau* inside the bulk, of those below the next step
outside it)."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, say
from oracle import rmt as ormt

pytestmark = pytest.mark.gpu
EIG_TOL = 1e-5


def gpu_csr(pairs, w, n):
    return sq.api.graph_topk(dev(pairs.astype(np.int32)), dev(w.astype(np.float32)), n, tau=0.0, k=0)


def family_graph(n, P, seed, fam_size=10):
    """Pairs from random_pairs with family structure; weights U(0.6, 1) within a family,
    U(0, 0.6) across (a stand-in for fused affinities, seeded)."""
    family = np.arange(n) // fam_size
    pairs = synth.random_pairs(n, P, seed, family=family, same_frac=0.5).astype(np.int64)
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    rng = np.random.default_rng(seed)
    same = family[pairs[:, 0]] == family[pairs[:, 1]]
    w = np.where(same, rng.uniform(0.6, 1.0, len(pairs)), rng.uniform(0.0, 0.6, len(pairs))).astype(np.float32)
    return pairs, w


def check_threshold(pairs, w, n, iters=ormt.ITERS):
    rows, cols, vals = gpu_csr(pairs, w, n)
    tau, lp, lmax = sq.api.rmt_threshold(rows, cols, vals, n, iters=iters)
    w64 = w.astype(np.float64)
    otau, olp, olmax, trace = ormt.threshold(pairs, w64, n, iters=iters, return_trace=True)
    assert lp == pytest.approx(olp, rel=1e-12)
    assert lmax == pytest.approx(olmax, rel=EIG_TOL)
    clear = all(abs(lm - olp) > 2 * EIG_TOL * max(lm, olp) for _, lm in trace)
    if clear and abs(olmax - olp) > 2 * EIG_TOL * olp:
        assert tau == otau, (tau, otau)
    elif olmax > olp:
        A = ormt.matrix(pairs, w64, n)
        step = A.data.max() * 2.0 ** -iters
        assert ormt.lambda_max(ormt.below(A, tau)) <= olp * (1 + 2 * EIG_TOL)
        assert ormt.lambda_max(ormt.below(A, tau + 1.0001 * step)) >= olp * (1 - 2 * EIG_TOL)
    return tau, otau


def test_planted_cliques():
    from test_oracle_rmt import _planted
    pairs, w, n, nclique = _planted()
    w = w.astype(np.float32)
    say(f"rmt planted cliques n={n}")
    tau, otau = check_threshold(pairs, w, n)
    assert tau == otau
    assert (w >= tau).sum() == nclique


def test_no_structure():
    from test_oracle_rmt import _planted
    pairs, w, n, _ = _planted(cliques=0)
    say("rmt no structure")
    rows, cols, vals = gpu_csr(pairs, w.astype(np.float32), n)
    tau, lp, lmax = sq.api.rmt_threshold(rows, cols, vals, n)
    assert lmax <= lp and tau > w.max()


@pytest.mark.parametrize("n,P,seed", [(2000, 12000, 1), (2500, 30000, 2), (20000, 80000, 3)])
def test_family_graphs(n, P, seed):
    pairs, w = family_graph(n, P, seed)
    say(f"rmt family graph n={n} P={len(pairs)}")
    check_threshold(pairs, w, n)


def test_lambda_max_of_masked_matrices():
    pairs, w = family_graph(3000, 20000, 4)
    n = 3000
    rows, cols, vals = gpu_csr(pairs, w, n)
    A = ormt.matrix(pairs, w.astype(np.float64), n)
    say("rmt masked lambda_max")
    for tau in (0.1, 0.35, 0.6, 0.8, float("inf")):
        got = sq.api.rmt_lambda_max(rows, cols, vals, n, tau=tau)
        ref = ormt.lambda_max(ormt.below(A, tau) if np.isfinite(tau) else A)
        assert got == pytest.approx(ref, rel=EIG_TOL, abs=1e-12), tau


def test_empty_and_tiny():
    say("rmt empty / one edge")
    rows, cols, vals = gpu_csr(np.zeros((0, 2), np.int64), np.zeros(0, np.float32), 10)
    tau, lp, lmax = sq.api.rmt_threshold(rows, cols, vals, 10)
    assert lp == 0.0 and lmax == 0.0 and tau == 1.0
    pairs = np.array([[0, 1]])
    w = np.array([0.75], np.float32)
    rows, cols, vals = gpu_csr(pairs, w, 2)
    tau, lp, lmax = sq.api.rmt_threshold(rows, cols, vals, 2)
    # one edge: lambda_max = w, lambda_plus = 2 sqrt(2 w^2 / 2) = 2 w > w: inside the bulk
    assert lmax == pytest.approx(0.75, rel=1e-6) and lp == pytest.approx(1.5, rel=1e-7) and tau > 0.75


def test_large_family_graph():
    """200,000 nodes, about 800,000 edges (the oracle's eigensolver is ARPACK here)."""
    pairs, w = family_graph(200_000, 800_000, 5)
    say(f"rmt family graph n=200000 P={len(pairs)}")
    check_threshold(pairs, w, 200_000)
