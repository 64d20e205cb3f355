"""Oracle: the paper's edit-distance affinity channel (Appendix F.3).

The recurrence is the weighted global edit distance
    d[x][y] = min(d[x-1][y] + del, d[x][y-1] + ins, d[x-1][y-1] + [a_x != b_y] * sub(a_x, b_y))
with insertion and deletion costs of one and a substitution cost "based on biochemical
similarity".  Reading (the paper gives no table): a substitution between residues with a
positive BLOSUM62 score (a conservative substitution) costs 1/2, any other substitution 1,
a match 0.  Costs are doubled so that the dynamic program runs in integers: indel 2,
conservative substitution 1, other substitution 2.  The affinity channel is
e_ij = 1 - d_ij / (2 max(L_i, L_j)), in [0, 1].
"""
from __future__ import annotations

import numpy as np

from .sw import _lib

INDEL = 2


def cost_matrix(subst) -> np.ndarray:
    """int8[20][20] doubled substitution costs from a substitution-score matrix."""
    S = np.asarray(subst, dtype=np.int64)
    C = np.where(S > 0, 1, 2).astype(np.int8)
    np.fill_diagonal(C, 0)
    return C


def distance_py(a, b, cost, indel=INDEL) -> int:
    la, lb = len(a), len(b)
    d = [[0] * (lb + 1) for _ in range(la + 1)]
    for x in range(la + 1):
        d[x][0] = x * indel
    for y in range(lb + 1):
        d[0][y] = y * indel
    for x in range(1, la + 1):
        for y in range(1, lb + 1):
            d[x][y] = min(d[x - 1][y] + indel, d[x][y - 1] + indel,
                          d[x - 1][y - 1] + int(cost[a[x - 1]][b[y - 1]]))
    return d[la][lb]


def distance_bruteforce(a, b, cost, indel=INDEL) -> int:
    """Minimum over every global alignment column sequence (tiny strings)."""
    from .sw import _alignments
    best = None
    for ops in _alignments(len(a), len(b)):
        x = y = 0
        tot = 0
        for op in ops:
            if op == "M":
                tot += int(cost[a[x]][b[y]])
                x += 1
                y += 1
            elif op == "I":
                tot += indel
                x += 1
            else:
                tot += indel
                y += 1
        best = tot if best is None else min(best, tot)
    return best


def distances_pairs(seqs, lens, pairs, cost, indel=INDEL) -> np.ndarray:
    """int32[P] doubled distances of the pairs (C loop)."""
    seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    C = np.ascontiguousarray(cost, dtype=np.int8)
    out = np.zeros(pairs.shape[0], dtype=np.int32)
    _lib().oracle_edit_pairs(seqs.ctypes.data, lens.ctypes.data, seqs.shape[1], pairs.ctypes.data,
                             pairs.shape[0], C.ctypes.data, indel, out.ctypes.data)
    return out


def similarity(dist, lens, pairs) -> np.ndarray:
    """e_ij = 1 - d_ij / (2 max(L_i, L_j)) (float64)."""
    L = np.asarray(lens, dtype=np.float64)
    p = np.asarray(pairs)
    return 1.0 - np.asarray(dist, dtype=np.float64) / (2.0 * np.maximum(L[p[:, 0]], L[p[:, 1]]))
