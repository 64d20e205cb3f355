"""Oracle: sparse similarity graph from the fused pair affinities.

Paper: Algorithm 1 (graph construction) builds A = [a~_ij] from the fused affinities and
keeps a sparse weighted graph G = (V, E, W) (Sec. 3.1 problem statement, Sec. 3.7); the
evaluation connects receptors whose fused similarity exceeds 0.7 (Sec. 4 network figure;
the sensitivity study of Appendix B places the best threshold at tau = 0.7) and reports
recall@k of the retrieved neighbours (Sec. 4 scalability).

Readings where the paper is silent:
  * the graph is undirected: a candidate pair (i, j) with fused weight w >= tau gives the
    edges i -> j and j -> i with weight w (pairs below tau, and non-candidates, give none);
  * each node's neighbours are ordered by weight descending, ties by neighbour id
    ascending, and the first k are kept (k = 0 keeps them all): the per-query top-k;
  * the result is CSR: row_offsets[n + 1], cols[nnz], vals[nnz].
The spectral (random-matrix) bulk cut-off of Sec. 3.7 is not part of this step.
"""
from __future__ import annotations

import numpy as np


def topk_graph(pairs, w, n: int, tau: float, k: int = 0):
    """(row_offsets int64[n+1], cols int32[nnz], vals float32[nnz]) -- weights compared as
    given (float32 in, float32 out)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(w, dtype=np.float32)
    keep = w >= np.float32(tau)
    i, j, ww = pairs[keep, 0], pairs[keep, 1], w[keep]
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    vals = np.concatenate([ww, ww])
    # order by (row, weight descending, neighbour ascending)
    order = np.lexsort((cols, -vals.astype(np.float64), rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    starts = np.searchsorted(rows, np.arange(n + 1), side="left")
    if k > 0:
        rank = np.arange(rows.shape[0]) - starts[rows]
        sel = rank < k
        rows, cols, vals = rows[sel], cols[sel], vals[sel]
        starts = np.searchsorted(rows, np.arange(n + 1), side="left")
    return starts.astype(np.int64), cols.astype(np.int32), vals.astype(np.float32)


def topk_graph_loops(pairs, w, n: int, tau: float, k: int = 0):
    """The same graph built node by node with Python lists (small inputs)."""
    adj = [[] for _ in range(n)]
    for (a, b), x in zip(np.asarray(pairs).tolist(), np.asarray(w, dtype=np.float32).tolist()):
        if x >= np.float32(tau):
            adj[a].append((x, b))
            adj[b].append((x, a))
    offs, cols, vals = [0], [], []
    for u in range(n):
        nb = sorted(adj[u], key=lambda t: (-t[0], t[1]))
        if k > 0:
            nb = nb[:k]
        cols += [v for _, v in nb]
        vals += [x for x, _ in nb]
        offs.append(len(cols))
    return np.array(offs, np.int64), np.array(cols, np.int32), np.array(vals, np.float32)


def recall_at_k(row_offsets, cols, family, k: int) -> float:
    """Mean over nodes with at least one other family member of
    |top-k neighbours in the same family| / min(k, family size - 1)."""
    family = np.asarray(family)
    sizes = np.bincount(family)
    rec = []
    for u in range(len(row_offsets) - 1):
        m = sizes[family[u]] - 1
        if m <= 0:
            continue
        nb = cols[row_offsets[u]:row_offsets[u + 1]][:k]
        rec.append(np.sum(family[nb] == family[u]) / min(k, m))
    return float(np.mean(rec)) if rec else 0.0
