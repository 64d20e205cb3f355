"""Seeded inputs besides the sequences: embeddings, gate weights, pair lists, gradients.

The paper computes per-sequence embeddings with a fine-tuned protein language encoder
(Sec. 3.2). No trained weights exist here, so embeddings are a seeded random projection of
each sequence's 3-mer count vector, L2-normalised (our reading). The projection matrix has
entries +1/-1 (an Achlioptas-style database-friendly projection) so that every projected
coordinate is a small integer and therefore exact in float32 on any device and in any
summation order; only the final normalisation rounds.
"""
from __future__ import annotations

import numpy as np
import torch

from .alphabet import PAD

N_3MERS = 8000


def _shingle_codes(seqs: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """int64[n][stride-2]: 400a+20b+c for every 3-mer position, N_3MERS past the end."""
    n, stride = seqs.shape
    s = seqs.astype(np.int64)
    s[s == PAD] = 0
    codes = 400 * s[:, :-2] + 20 * s[:, 1:-1] + s[:, 2:]
    pos = np.arange(stride - 2)[None, :]
    codes[pos + 3 > lens[:, None].astype(np.int64)] = N_3MERS
    return codes


def projection_matrix(d: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    R = (rng.integers(0, 2, (N_3MERS, d)) * 2 - 1).astype(np.float32)
    return np.concatenate([R, np.zeros((1, d), np.float32)])


def embeddings(seqs: np.ndarray, lens: np.ndarray, d: int, seed: int = 4242,
               device: str = "cpu", chunk: int = 1 << 20):
    """float32[n][d] unit embeddings. Returns a numpy array (cpu) or a torch tensor."""
    R = torch.from_numpy(projection_matrix(d, seed)).to(device)
    n = seqs.shape[0]
    out = torch.empty((n, d), dtype=torch.float32, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        codes = torch.from_numpy(_shingle_codes(seqs[lo:hi], lens[lo:hi])).to(device)
        v = torch.nn.functional.embedding_bag(codes, R, mode="sum", padding_idx=N_3MERS)
        ss = (v.double() ** 2).sum(1, keepdim=True)
        # a zero projection (possible for small d) stays the zero vector
        out[lo:hi] = (v.double() / torch.sqrt(torch.where(ss > 0, ss, torch.ones_like(ss)))).float()
    return out.numpy() if device == "cpu" else out


def gate_params(H: int = 64, seed: int = 77):
    """Gate MLP weights 4 -> H -> 1 with the usual U(+-1/sqrt(fan_in)) initialisation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a1 = 1.0 / np.sqrt(4.0)
    a2 = 1.0 / np.sqrt(H)
    W1 = rng.uniform(-a1, a1, (H, 4)).astype(np.float32)
    b1 = rng.uniform(-a1, a1, H).astype(np.float32)
    w2 = rng.uniform(-a2, a2, H).astype(np.float32)
    b2 = rng.uniform(-a2, a2, 1).astype(np.float32)
    return W1, b1, w2, b2


def random_pairs(n: int, P: int, seed: int, family=None, same_frac: float = 0.5,
                 rep_offsets=None) -> np.ndarray:
    """int32[P'][2] distinct pairs i<j sorted by (i, j), P' <= P.

    About ``same_frac`` of them join members of one family (when ``family`` is given), the
    rest are uniform; with ``rep_offsets`` no pair crosses repertoires.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    if family is not None and same_frac > 0:
        order = np.argsort(family, kind="stable")
        fam_sorted = family[order]
        starts = np.searchsorted(fam_sorted, fam_sorted, side="left")
        ends = np.searchsorted(fam_sorted, fam_sorted, side="right")
        m = int(P * same_frac)
        a = rng.integers(0, n, m)
        pa = np.argsort(order)[a]
        size = ends[pa] - starts[pa]
        ok = size > 1
        off = rng.integers(0, np.maximum(size, 1))
        b = order[starts[pa] + off]
        sel = ok & (b != a)
        out.append(np.stack([a[sel], b[sel]], 1))
    m = P - (out[0].shape[0] if out else 0)
    if rep_offsets is None or len(rep_offsets) <= 2:
        a = rng.integers(0, n, m)
        b = rng.integers(0, n, m)
    else:
        offs = np.asarray(rep_offsets)
        sizes = np.diff(offs)
        r = rng.choice(len(sizes), m, p=sizes / sizes.sum())
        a = offs[r] + rng.integers(0, sizes[r])
        b = offs[r] + rng.integers(0, sizes[r])
    sel = a != b
    out.append(np.stack([a[sel], b[sel]], 1))
    pr = np.concatenate(out).astype(np.int64)
    pr.sort(axis=1)
    key = np.unique(pr[:, 0] * n + pr[:, 1])
    return np.stack([key // n, key % n], 1).astype(np.int32)


def upstream_grad(P: int, seed: int = 99) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(P).astype(np.float32)


def sample_rows(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)
