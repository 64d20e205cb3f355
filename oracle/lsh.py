"""Oracle: MinHash LSH banding into candidate pairs.

Paper: Algorithm 1 (preprocessing) builds a MinHash LSH index and generates the candidate
list CAND for each query; Sec. 4.2 describes the index; Appendix B.2 puts the cost of
retrieval at O(|C|) + O(n log n) with C the candidate set.

Readings where the paper is silent:
  * standard b x r banding with contiguous rows: band beta covers signature rows
    beta*r .. beta*r + r - 1, and b*r <= M (rows past b*r are unused);
  * a pair (i, j), i < j, is a candidate iff for at least one band the two r-tuples are
    EXACTLY equal (no hash of the band stands in for the tuple);
  * the candidate set is a set (a pair matching in several bands appears once), has no
    self-pairs, never crosses repertoires, and is listed sorted by (i, j);
  * buckets have no size cap.
"""
from __future__ import annotations

import numpy as np


def rep_ids(n: int, rep_offsets=None) -> np.ndarray:
    if rep_offsets is None:
        return np.zeros(n, dtype=np.int64)
    offs = np.asarray(rep_offsets, dtype=np.int64)
    return np.searchsorted(offs, np.arange(n), side="right") - 1


def candidates(sig: np.ndarray, b: int, r: int, rep_offsets=None) -> np.ndarray:
    """int64[P][2] candidate pairs by grouping equal band tuples (plain Python dicts)."""
    n, M = sig.shape
    if b * r > M:
        raise ValueError("b*r exceeds the signature length")
    rep = rep_ids(n, rep_offsets)
    found = set()
    for beta in range(b):
        groups: dict = {}
        block = sig[:, beta * r:(beta + 1) * r]
        for i in range(n):
            key = (int(rep[i]),) + tuple(int(v) for v in block[i])
            groups.setdefault(key, []).append(i)
        for ids in groups.values():
            for x in range(len(ids)):
                for y in range(x + 1, len(ids)):
                    found.add((ids[x], ids[y]))
    if not found:
        return np.zeros((0, 2), dtype=np.int64)
    return np.array(sorted(found), dtype=np.int64)


def candidates_bruteforce(sig: np.ndarray, b: int, r: int, rep_offsets=None) -> np.ndarray:
    """The definition checked over every pair i < j (O(n^2 b)); small n only."""
    n = sig.shape[0]
    rep = rep_ids(n, rep_offsets)
    bands = sig[:, : b * r].reshape(n, b, r)
    out = []
    for i in range(n):
        eq = (bands[i + 1:] == bands[i][None]).all(axis=2).any(axis=1)
        eq &= rep[i + 1:] == rep[i]
        for j in np.nonzero(eq)[0]:
            out.append((i, i + 1 + int(j)))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def candidates_of_row(sig: np.ndarray, i: int, b: int, r: int, rep_offsets=None) -> np.ndarray:
    """Sorted j > i that form a candidate with i (vectorised over j; any n)."""
    n = sig.shape[0]
    rep = rep_ids(n, rep_offsets)
    hi = n
    if rep_offsets is not None:
        hi = int(np.asarray(rep_offsets)[rep[i] + 1])
    bands = sig[i + 1:hi, : b * r].reshape(-1, b, r)
    eq = (bands == sig[i, : b * r].reshape(b, r)[None]).all(axis=2).any(axis=1)
    return (i + 1 + np.nonzero(eq)[0]).astype(np.int64)


def candidates_grouped(sig: np.ndarray, b: int, r: int, rep_offsets=None,
                       max_visits: int = 200_000_000) -> np.ndarray:
    """Same set as :func:`candidates`, built with numpy grouping (for larger n whose
    buckets are small). Raises if the buckets would yield more than ``max_visits`` pairs."""
    n = sig.shape[0]
    rep = rep_ids(n, rep_offsets).astype(np.uint64)
    keys = []
    for beta in range(b):
        rows = np.concatenate([rep[:, None], sig[:, beta * r:(beta + 1) * r]], axis=1)
        v = np.ascontiguousarray(rows).view(np.dtype((np.void, 8 * (r + 1)))).ravel()
        _, inv, cnt = np.unique(v, return_inverse=True, return_counts=True)
        order = np.argsort(inv, kind="stable")          # members of a group, ascending id
        g = inv[order]
        start = np.searchsorted(g, g, side="left")
        end = np.searchsorted(g, g, side="right")
        pos = np.arange(n)
        later = end - pos - 1                           # members after this one
        if int(later.sum()) > max_visits:
            raise MemoryError("buckets too large for the grouped oracle")
        src = np.repeat(pos, later)
        first = np.repeat(pos + 1 - np.concatenate([[0], np.cumsum(later)[:-1]]), later)
        dst = first + np.arange(src.shape[0])
        i_ids = order[src].astype(np.int64)
        j_ids = order[dst].astype(np.int64)
        del start
        lo = np.minimum(i_ids, j_ids)
        hi = np.maximum(i_ids, j_ids)
        keys.append(lo * n + hi)
    allk = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    return np.stack([allk // n, allk % n], axis=1)


def collision_probability(J: float, b: int, r: int) -> float:
    """Probability that a pair of Jaccard index J shares at least one band under ideal
    min-wise hashing: 1 - (1 - J^r)^b."""
    return 1.0 - (1.0 - J ** r) ** b
