"""Oracle: 3-mer shingles and 64-bit MinHash signatures.

Paper: Algorithm 1 (preprocessing) computes MinHash sketches of every sequence; Appendix B
(MinHash prefiltering, sampling-error bounds) fixes the sketch size M and the 1/sqrt(M)
error scale of the Jaccard estimate; Sec. 4.1 sweeps M over {64, 128, 256}.

Readings where the paper is silent:
  * shingles are the SET of distinct contiguous 3-mers (a, b, c) of a sequence;
  * hash t < M is simple tabulation over the three positions,
        h_t(a, b, c) = T[t][0][a] xor T[t][1][b] xor T[t][2][c]   (64-bit),
    whose 60*M table words are consecutive outputs of SplitMix64 (Steele, Lea & Flood,
    OOPSLA 2014) started from ``seed``, taken in the order t, then position, then residue;
  * the signature is sig[t] = min over shingles x of h_t(x), as an unsigned 64-bit value.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of SplitMix64 from state ``seed`` (pure Python ints).

    Each step adds the golden-ratio increment to the state and returns the state passed
    through the variant-13 finaliser (shift 30, multiply, shift 27, multiply, shift 31).
    """
    out = []
    x = seed & MASK64
    for _ in range(count):
        x = (x + GOLDEN_GAMMA) & MASK64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def hash_tables(seed: int, M: int) -> np.ndarray:
    """uint64[M][3][20]: the tabulation words, in SplitMix64 output order."""
    vals = splitmix64(seed, M * 3 * 20)
    return np.array(vals, dtype=np.uint64).reshape(M, 3, 20)


def shingles(codes) -> set:
    """The set of contiguous 3-mers of a residue-code sequence."""
    codes = [int(c) for c in codes]
    return {(codes[p], codes[p + 1], codes[p + 2]) for p in range(len(codes) - 2)}


def hash3(T: np.ndarray, t: int, a: int, b: int, c: int) -> int:
    return int(T[t, 0, a]) ^ int(T[t, 1, b]) ^ int(T[t, 2, c])


def signature(codes, T: np.ndarray) -> np.ndarray:
    """sig[t] = min over the shingle set of h_t (pure Python; small inputs)."""
    sh = shingles(codes)
    if not sh:
        raise ValueError("a sequence needs at least 3 residues")
    M = T.shape[0]
    return np.array([min(hash3(T, t, *x) for x in sh) for t in range(M)], dtype=np.uint64)


def signatures(seqs: np.ndarray, lens: np.ndarray, M: int, seed: int) -> np.ndarray:
    """uint64[n][M] for a whole padded batch (numpy, vectorised over sequences).

    The minimum over the shingle set equals the minimum over shingle positions, since a
    repeated 3-mer contributes the same hash value again; positions past a sequence's end
    are excluded.
    """
    T = hash_tables(seed, M)
    n, stride = seqs.shape
    lens = np.asarray(lens, dtype=np.int64)
    if n and lens.min() < 3:
        raise ValueError("a sequence needs at least 3 residues")
    s = seqs.astype(np.int64)
    s[s >= 20] = 0
    sig = np.full((n, M), np.iinfo(np.uint64).max, dtype=np.uint64)
    for p in range(stride - 2):
        live = lens >= p + 3
        if not live.any():
            break
        rows = np.nonzero(live)[0]
        h = T[:, 0, s[rows, p]] ^ T[:, 1, s[rows, p + 1]] ^ T[:, 2, s[rows, p + 2]]
        sig[rows] = np.minimum(sig[rows], h.T)
    return sig


def jaccard(codes_a, codes_b) -> float:
    """Exact Jaccard index of two shingle sets."""
    A, B = shingles(codes_a), shingles(codes_b)
    return len(A & B) / len(A | B)


def jaccard_estimate(sig_a: np.ndarray, sig_b: np.ndarray) -> float:
    """Fraction of hash functions on which two signatures agree."""
    return float(np.mean(sig_a == sig_b))


def signatures_c(seqs: np.ndarray, lens: np.ndarray, M: int, seed: int) -> np.ndarray:
    """Same as :func:`signatures`, computed by the plain C loop in ``minhash_ref.c``."""
    from .sw import _lib
    T = np.ascontiguousarray(hash_tables(seed, M))
    seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    if lens.size and (lens.min() < 3 or lens.max() > seqs.shape[1]):
        raise ValueError("lengths must lie in [3, stride]")
    if seqs.size and (seqs[np.arange(seqs.shape[1])[None, :] < lens[:, None]] >= 20).any():
        raise ValueError("residue codes must be below 20")
    out = np.zeros((seqs.shape[0], M), dtype=np.uint64)
    _lib().oracle_minhash3(seqs.ctypes.data, lens.ctypes.data, seqs.shape[0], seqs.shape[1],
                           T.ctypes.data, M, out.ctypes.data)
    return out
