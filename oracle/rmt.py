"""Oracle: random-matrix-theory edge threshold for the similarity graph, float64.
TEST INFRASTRUCTURE ONLY.

Paper: Sec. 3.7 (graph construction and RMT-based thresholding) and Algorithm 1: build the
symmetric similarity matrix A of fused affinities, take its eigenvalue spectrum, estimate
the cutoff of the noise bulk, and drop the edges whose weights fall below the threshold that
cutoff implies.  The paper names no estimator; readings taken here:

  * A: a_ij = a_ji = max(f_ij, 0) for every candidate pair (i, j) with a finite affinity
    (negative affinities make no edge), zero diagonal, zero elsewhere;
  * bulk cutoff: the edge of the Wigner semicircle of a symmetric random matrix with the same
    mean squared row norm, lambda_plus = 2 sqrt(sum_ij a_ij^2 / n);
  * threshold: the edges lighter than tau form A_low(tau) (0 < a_ij < tau).  Since A >= 0,
    the largest eigenvalue of A_low(tau) grows with tau (Perron-Frobenius).  tau* is the
    largest tau for which A_low(tau) stays inside the bulk, lambda_max(A_low(tau)) <=
    lambda_plus: those edges are indistinguishable from noise, the heavier ones carry the
    eigenvalues outside the bulk.  tau* is found by `iters` bisection steps on [0, max a_ij]
    with float64 midpoints; edges with a_ij >= tau* are kept.  When even the whole matrix
    stays inside the bulk there is no structure: tau* = max a_ij + 1 and no edge is kept.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

ITERS = 20
DENSE_LIMIT = 3000


def matrix(pairs, w, n):
    """Symmetric scipy CSR matrix A (float64) of the positive finite affinities."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(w, dtype=np.float64)
    keep = np.isfinite(w) & (w > 0) & (pairs[:, 0] != pairs[:, 1])
    i, j, v = pairs[keep, 0], pairs[keep, 1], w[keep]
    A = sp.coo_matrix((np.concatenate([v, v]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))
    return A.tocsr()


def bulk_edge(A) -> float:
    """lambda_plus = 2 sqrt(sum a_ij^2 / n)."""
    n = A.shape[0]
    return 2.0 * float(np.sqrt((A.data.astype(np.float64) ** 2).sum() / max(n, 1)))


def lambda_max(A) -> float:
    """Largest eigenvalue of a symmetric matrix (0 for an empty one)."""
    if A.nnz == 0:
        return 0.0
    n = A.shape[0]
    if n <= DENSE_LIMIT:
        return float(np.linalg.eigvalsh(A.toarray())[-1])
    return float(spla.eigsh(A.astype(np.float64), k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0])


def below(A, tau):
    """A_low(tau): the entries with 0 < a_ij < tau."""
    B = A.copy()
    B.data = np.where(B.data < tau, B.data, 0.0)
    B.eliminate_zeros()
    return B


def threshold(pairs, w, n, iters: int = ITERS, return_trace: bool = False):
    """(tau*, lambda_plus, lambda_max(A)) by bisection; with return_trace also the list of
    (tau, lambda_max(A_low(tau))) of every step."""
    A = matrix(pairs, w, n)
    lp = bulk_edge(A)
    lmax = lambda_max(A)
    wmax = float(A.data.max()) if A.nnz else 0.0
    trace = []
    if lmax <= lp:
        tau = wmax + 1.0
    else:
        lo, hi = 0.0, wmax
        # A_low(wmax) lacks only the heaviest edges; if it still exceeds the bulk the answer
        # is below wmax, which the bisection finds; lambda_max(A_low(0)) = 0 <= lp always.
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            lm = lambda_max(below(A, mid))
            trace.append((mid, lm))
            if lm <= lp:
                lo = mid
            else:
                hi = mid
        tau = lo
    return (tau, lp, lmax, trace) if return_trace else (tau, lp, lmax)


def tridiag_eigvals(alpha, beta):
    """Eigenvalues of the symmetric tridiagonal matrix with diagonal alpha and off-diagonal
    beta (a Lanczos T_k), ascending."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    return np.linalg.eigvalsh(T)
