"""Oracle: Smith-Waterman local alignment score (Gotoh, affine gaps) and self-scores.

The dynamic program itself is plain C in ``sw_ref.c`` (full matrices, textbook order);
this module builds and loads it, and adds a pure-Python version of the same recurrence
and an exhaustive enumeration of alignments used to pin both on tiny strings.

Gap convention (reading): a gap of length k costs gap_open + (k - 1) * gap_extend.
Self-score (reading of the normalised score): S_i = sum over x of subst[a_x][a_x], which
equals SW(a, a) whenever every off-diagonal entry of the matrix is below every diagonal
entry (true of BLOSUM62).
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "sw_ref.c"), os.path.join(_HERE, "minhash_ref.c")]
_LIB = os.path.join(_HERE, "_oracle_ref.so")


def build(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc into ``oracle/_oracle_ref.so``."""
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=1)
def _lib():
    lib = ctypes.CDLL(build())
    lib.oracle_sw_score.restype = ctypes.c_int
    lib.oracle_sw_score.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.oracle_minhash3.restype = None
    lib.oracle_minhash3.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    lib.oracle_edit_pairs.restype = None
    lib.oracle_edit_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.oracle_sw_pairs.restype = None
    lib.oracle_sw_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    return lib


def score_c(a, b, subst, gap_open=10, gap_extend=1) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    S = np.ascontiguousarray(subst, dtype=np.int8)
    return _lib().oracle_sw_score(a.ctypes.data, a.size, b.ctypes.data, b.size,
                                  S.ctypes.data, gap_open, gap_extend)


def scores_pairs(seqs, lens, pairs, subst, gap_open=10, gap_extend=1) -> np.ndarray:
    """int32[P]: SW score of every pair (i, j) of rows of ``seqs`` (C, one thread)."""
    seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    S = np.ascontiguousarray(subst, dtype=np.int8)
    out = np.zeros(pairs.shape[0], dtype=np.int32)
    _lib().oracle_sw_pairs(seqs.ctypes.data, lens.ctypes.data, seqs.shape[1], pairs.ctypes.data,
                           pairs.shape[0], S.ctypes.data, gap_open, gap_extend, out.ctypes.data)
    return out


_SHARED: dict = {}


def _pool_chunk(k):
    d = _SHARED
    return scores_pairs(d["seqs"], d["lens"], d["chunks"][k], d["subst"], d["go"], d["ge"])


def scores_pairs_parallel(seqs, lens, pairs, subst, gap_open=10, gap_extend=1, procs=None):
    """Same as :func:`scores_pairs`, split over worker processes (CPU baseline timing).

    The tables reach the workers through the fork (module globals set before the pool
    starts), so a task carries only its chunk index."""
    import multiprocessing as mp
    procs = procs or len(os.sched_getaffinity(0))
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    build()
    _SHARED.update(seqs=np.ascontiguousarray(seqs, dtype=np.uint8), lens=np.ascontiguousarray(lens, dtype=np.int32),
                   chunks=np.array_split(pairs, procs * 4), subst=np.ascontiguousarray(subst, dtype=np.int8),
                   go=gap_open, ge=gap_extend)
    try:
        with mp.get_context("fork").Pool(procs) as pool:
            parts = pool.map(_pool_chunk, range(len(_SHARED["chunks"])))
    finally:
        _SHARED.clear()
    return np.concatenate(parts) if parts else np.zeros(0, np.int32)


def score_py(a, b, subst, gap_open=10, gap_extend=1) -> int:
    """Gotoh's recurrence in pure Python (same definition as ``sw_ref.c``)."""
    NEG = -10**9
    la, lb = len(a), len(b)
    H = [[0] * (lb + 1) for _ in range(la + 1)]
    E = [[NEG] * (lb + 1) for _ in range(la + 1)]
    F = [[NEG] * (lb + 1) for _ in range(la + 1)]
    best = 0
    for x in range(1, la + 1):
        for y in range(1, lb + 1):
            E[x][y] = max(E[x][y - 1] - gap_extend, H[x][y - 1] - gap_open)
            F[x][y] = max(F[x - 1][y] - gap_extend, H[x - 1][y] - gap_open)
            H[x][y] = max(0, H[x - 1][y - 1] + int(subst[a[x - 1]][b[y - 1]]), E[x][y], F[x][y])
            best = max(best, H[x][y])
    return best


@functools.lru_cache(maxsize=None)
def _alignments(m: int, n: int) -> tuple:
    """Every column sequence aligning m residues of a with n of b.
    'M' pairs a residue of each, 'I' consumes a only, 'D' consumes b only."""
    if m == 0 and n == 0:
        return ("",)
    out = []
    if m and n:
        out += ["M" + s for s in _alignments(m - 1, n - 1)]
    if m:
        out += ["I" + s for s in _alignments(m - 1, n)]
    if n:
        out += ["D" + s for s in _alignments(m, n - 1)]
    return tuple(out)


def alignment_score(a, b, ops: str, subst, gap_open, gap_extend) -> int:
    """Score of one explicit alignment: substitution scores of 'M' columns minus, for
    every maximal run of k equal gap columns, gap_open + (k - 1) * gap_extend."""
    x = y = 0
    total = 0
    prev = ""
    for op in ops:
        if op == "M":
            total += int(subst[a[x]][b[y]])
            x += 1
            y += 1
        elif op == "I":
            total -= gap_extend if prev == "I" else gap_open
            x += 1
        else:
            total -= gap_extend if prev == "D" else gap_open
            y += 1
        prev = op
    return total


def score_bruteforce(a, b, subst, gap_open=10, gap_extend=1) -> int:
    """Best score over every alignment of every pair of substrings (and 0 for the empty
    alignment). Exponential: strings of length <= 5 or so."""
    best = 0
    for i1 in range(len(a)):
        for i2 in range(i1 + 1, len(a) + 1):
            for j1 in range(len(b)):
                for j2 in range(j1 + 1, len(b) + 1):
                    sa, sb = a[i1:i2], b[j1:j2]
                    for ops in _alignments(len(sa), len(sb)):
                        best = max(best, alignment_score(sa, sb, ops, subst, gap_open, gap_extend))
    return best


def self_scores(seqs, lens, subst) -> np.ndarray:
    """int32[n]: sum of diagonal substitution scores along each sequence."""
    seqs = np.asarray(seqs)
    diag = np.diag(np.asarray(subst, dtype=np.int64))
    s = seqs.astype(np.int64)
    live = np.arange(seqs.shape[1])[None, :] < np.asarray(lens)[:, None]
    return np.where(live, diag[np.where(live, s, 0)], 0).sum(axis=1).astype(np.int32)
