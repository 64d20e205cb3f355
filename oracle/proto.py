"""Oracle: prototype-contrastive loss and its gradient, float64.  TEST INFRASTRUCTURE ONLY.

Paper: Sec. 3 (prototype-contrastive consolidation), Eq. (pc) and Eq. (proto):
  p_c = mean of f(x) over the examples S_c with label c;
  L   = - sum over the batch B of log( exp(<f(x), p_y(x)> / tau) / sum_{c' in N_x} exp(<f(x), p_c'> / tau) ).

Readings where the paper is silent:
  * f(x) is a row of the embedding table E[n][d] (the same table the gate's cosine channel
    reads); S_c is every row of the table with label c, so the prototypes are recomputed
    from the current table;
  * N_x is every non-empty class, the positive one included (the softmax form, so each term
    is a log-probability and L >= 0); classes with no example have no prototype and are left
    out;
  * the batch B is a list of row indices (repeats allowed), the loss is the sum over it;
  * tau = 0.1 unless given;
  * the gradient reaches E along two routes: through f(x) for x in B, and, because Eq. (pc)
    makes every prototype a function of the table, through p_c into every row of S_c.
    ``through_prototypes=False`` treats the prototypes as constants instead (a maintained,
    detached prototype bank).
"""
from __future__ import annotations

import numpy as np

TAU = 0.1


def prototypes(emb, labels, C: int):
    """(P[C][d] class means, counts[C]) in float64; rows of empty classes are zero."""
    E = np.asarray(emb, dtype=np.float64)
    y = np.asarray(labels, dtype=np.int64)
    counts = np.bincount(y, minlength=C).astype(np.int64)
    sums = np.zeros((C, E.shape[1]))
    np.add.at(sums, y, E)
    P = sums / np.maximum(counts, 1)[:, None]
    return P, counts


def logits(emb, labels, batch, C: int, tau: float = TAU):
    """(Z[B][C] = <f(x), p_c> / tau with empty classes at -inf, P, counts)."""
    P, counts = prototypes(emb, labels, C)
    F = np.asarray(emb, dtype=np.float64)[np.asarray(batch, dtype=np.int64)]
    Z = F @ P.T / tau
    Z[:, counts == 0] = -np.inf
    return Z, P, counts


def loss(emb, labels, batch, C: int, tau: float = TAU, return_rows: bool = False):
    """Eq. (proto): sum over the batch of logsumexp_c Z[x][c] - Z[x][y(x)]."""
    Z, _, _ = logits(emb, labels, batch, C, tau)
    yb = np.asarray(labels, dtype=np.int64)[np.asarray(batch, dtype=np.int64)]
    m = Z.max(axis=1)
    lse = m + np.log(np.exp(Z - m[:, None]).sum(axis=1))
    rows = lse - Z[np.arange(Z.shape[0]), yb]
    return (float(rows.sum()), rows, lse) if return_rows else float(rows.sum())


def backward(emb, labels, batch, C: int, tau: float = TAU, grad_loss: float = 1.0,
             through_prototypes: bool = True):
    """dE[n][d] = grad_loss * dL/dE (float64)."""
    E = np.asarray(emb, dtype=np.float64)
    b = np.asarray(batch, dtype=np.int64)
    y = np.asarray(labels, dtype=np.int64)
    Z, P, counts = logits(E, y, b, C, tau)
    m = Z.max(axis=1, keepdims=True)
    pi = np.exp(Z - m)
    pi /= pi.sum(axis=1, keepdims=True)                 # softmax over the classes
    G = pi.copy()
    G[np.arange(len(b)), y[b]] -= 1.0                    # dL/dZ
    G *= grad_loss / tau                                 # dL/d<f, p>
    dE = np.zeros_like(E)
    np.add.at(dE, b, G @ P)                              # through f(x), x in B
    if through_prototypes:
        dP = G.T @ E[b]                                  # dL/dp_c
        dE += dP[y] / np.maximum(counts[y], 1)[:, None]  # through p_c = mean over S_c
    return dE
