"""Seeded synthetic CDR3 repertoires shaped like the paper's workloads.

The paper evaluates on CDR3-beta repertoires (VDJdb, McPAS-TCR and others, Appendix
configuration table). Those datasets are not available here, so every workload is a
synthetic stand-in with the same structure: clonotype families grown from random seed
sequences by point substitutions and at most one indel, with skewed family sizes,
V-gene labels and a rare subgroup. All randomness comes from
``numpy.random.Generator(PCG64(seed))``; the same seed gives the same arrays on any
machine. This module holds none of the method's arithmetic.

Member recipe (our reading; the paper gives no generator):
  * a seed has length U{Lmin..Lmax} and uniform residues;
  * a member copies its family's seed, applies k ~ U{0..kmax} substitutions at distinct
    positions (each to one of the 19 other letters), then with probability ``p_indel``
    one insertion or deletion (1/2 each) at a uniform position; an indel that would leave
    [Lmin, Lmax] is flipped;
  * member 0 of every family is the seed itself, and sequences are unique within a
    repertoire (a duplicate is redrawn);
  * the final order of sequences is a seeded random permutation, so families are not
    contiguous in memory.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .alphabet import PAD

N_VGENES = 48


@dataclass
class Repertoire:
    """A batch of one or more repertoires, concatenated.

    ``rep_offsets[r]:rep_offsets[r+1]`` is repertoire ``r``. ``family`` ids are global
    (unique across repertoires).
    """

    name: str
    seqs: np.ndarray          # uint8[n][stride], PAD past the length
    lens: np.ndarray          # int32[n]
    family: np.ndarray        # int32[n]
    vgene: np.ndarray         # int32[n]
    subgroup: np.ndarray      # int8[n], 1 = rare subgroup
    rep_offsets: np.ndarray   # int64[R+1]
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.lens.shape[0])

    @property
    def stride(self) -> int:
        return int(self.seqs.shape[1])


def _zipf_probs(k: int, s: float = 1.5) -> np.ndarray:
    w = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def _random_seeds(rng, F, Lmin, Lmax, stride):
    lens = rng.integers(Lmin, Lmax + 1, F).astype(np.int32)
    codes = rng.integers(0, 20, (F, stride)).astype(np.uint8)
    codes[np.arange(stride)[None, :] >= lens[:, None]] = PAD
    return codes, lens


def _mutate(rng, seed_codes, seed_lens, fam, kmax, p_indel, Lmin, Lmax):
    """Members of families ``fam`` (one row per entry of ``fam``)."""
    N = fam.shape[0]
    stride = seed_codes.shape[1]
    codes = seed_codes[fam].copy()
    L = seed_lens[fam].astype(np.int64)
    col = np.arange(stride)[None, :]
    # substitutions at k distinct positions
    k = rng.integers(0, kmax + 1, N)
    keys = rng.random((N, stride))
    keys[col >= L[:, None]] = 2.0
    order = np.argsort(keys, axis=1, kind="stable")
    for s in range(kmax):
        rows = np.nonzero(k > s)[0]
        if rows.size == 0:
            continue
        pos = order[rows, s]
        shift = rng.integers(1, 20, rows.size)
        codes[rows, pos] = ((codes[rows, pos].astype(np.int64) + shift) % 20).astype(np.uint8)
    # at most one indel
    has = rng.random(N) < p_indel
    ins = rng.random(N) < 0.5
    ins = np.where(L >= Lmax, False, np.where(L <= Lmin, True, ins))
    rows = np.nonzero(has & ins)[0]
    if rows.size:
        p = rng.integers(0, L[rows] + 1)
        res = rng.integers(0, 20, rows.size).astype(np.uint8)
        src = np.clip(np.where(col < p[:, None], col, col - 1), 0, stride - 1)
        new = np.take_along_axis(codes[rows], src, axis=1)
        hit = col == p[:, None]
        new[hit] = np.repeat(res, hit.sum(axis=1))
        Lr = L[rows] + 1
        new[col >= Lr[:, None]] = PAD
        codes[rows] = new
        L[rows] = Lr
    rows = np.nonzero(has & ~ins)[0]
    if rows.size:
        p = rng.integers(0, L[rows])
        src = np.clip(np.where(col < p[:, None], col, col + 1), 0, stride - 1)
        new = np.take_along_axis(codes[rows], src, axis=1)
        Lr = L[rows] - 1
        new[col >= Lr[:, None]] = PAD
        codes[rows] = new
        L[rows] = Lr
    return codes, L.astype(np.int32)


def _dup_mask(codes):
    """True for rows equal to an earlier row."""
    v = np.ascontiguousarray(codes).view(np.dtype((np.void, codes.shape[1]))).ravel()
    _, first = np.unique(v, return_index=True)
    mask = np.ones(codes.shape[0], dtype=bool)
    mask[first] = False
    return mask


def families_to_repertoire(rng, sizes, Lmin, Lmax, kmax, p_indel, stride=32):
    """Grow families of the given sizes; returns (codes, lens, family) in shuffled order."""
    sizes = np.asarray(sizes, dtype=np.int64)
    F = sizes.shape[0]
    seed_codes, seed_lens = _random_seeds(rng, F, Lmin, Lmax, stride)
    fam = np.repeat(np.arange(F, dtype=np.int64), sizes)
    first = np.zeros(fam.shape[0], dtype=bool)
    first[np.concatenate([[0], np.cumsum(sizes)[:-1]])] = True
    codes, lens = _mutate(rng, seed_codes, seed_lens, fam, kmax, p_indel, Lmin, Lmax)
    codes[first] = seed_codes
    lens[first] = seed_lens
    for _ in range(1000):
        dup = _dup_mask(codes)
        if not dup.any():
            break
        rows = np.nonzero(dup)[0]
        c2, l2 = _mutate(rng, seed_codes, seed_lens, fam[rows], kmax, p_indel, Lmin, Lmax)
        codes[rows] = c2
        lens[rows] = l2
    else:  # pragma: no cover - a family too small to hold unique members
        raise RuntimeError("could not make sequences unique")
    perm = rng.permutation(fam.shape[0])
    return codes[perm], lens[perm], fam[perm].astype(np.int32)


def _vgenes_for_families(rng, F):
    return rng.choice(N_VGENES, size=F, p=_zipf_probs(N_VGENES)).astype(np.int32)


def zipf_rank_sizes(total: int, F: int, s: float = 1.5) -> np.ndarray:
    """Family sizes proportional to rank^-s, at least 1, summing exactly to ``total``.

    A scale is found so that sum(max(1, scale * w_k)) = total; the fractional parts of the
    families above 1 are then apportioned by largest remainder.
    """
    w = np.arange(1, F + 1, dtype=np.float64) ** (-s)
    lo, hi = 0.0, float(total) / w[-1]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.maximum(1.0, mid * w).sum() > total:
            hi = mid
        else:
            lo = mid
    q = np.maximum(1.0, lo * w)
    base = np.floor(q).astype(np.int64)
    rem = total - int(base.sum())
    frac = q - base
    frac[q <= 1.0] = -1.0
    base[np.argsort(-frac, kind="stable")[:rem]] += 1
    assert base.sum() == total and base.min() >= 1
    return base


# --------------------------------------------------------------------------- configs
#
# Workloads named by what they are. Seeds are 1000 + the workload's ordinal.
#   small5k   : 5,000 sequences, 500 families x 10, lengths 8-20, M=64, 16x4 bands, d=64
#   zipf100k  : 100,000 sequences from 10,000 rank-Zipf(1.5) families, lengths 8-25,
#               M=128, 32x4, d=128
#   rep1m     : 1,000,000 sequences, 100,000 families (2,000 rare families of 1-3
#               members), lengths 8-20, M=128, 32x4, d=128
#   batch64   : 64 repertoires of log-uniform size 1e4..2e6, lengths 8-30, i.i.d.
#               Zipf(1.5) family sizes truncated to [1, 1000]

WORKLOADS = {
    "small5k": dict(seed=1001, Lmin=8, Lmax=20, kmax=3, p_indel=0.1, M=64, b=16, r=4, d=64),
    "zipf100k": dict(seed=1002, Lmin=8, Lmax=25, kmax=4, p_indel=0.1, M=128, b=32, r=4, d=128),
    "rep1m": dict(seed=1003, Lmin=8, Lmax=20, kmax=3, p_indel=0.1, M=128, b=32, r=4, d=128),
    "batch64": dict(seed=1005, Lmin=8, Lmax=30, kmax=3, p_indel=0.1, M=128, b=32, r=4, d=128),
}
HASH_SEED = 260217330
GATE_HIDDEN = 64


def _finish(name, codes, lens, fam, fam_vgene, fam_rare, rep_offsets, params):
    return Repertoire(
        name=name,
        seqs=codes,
        lens=lens,
        family=fam,
        vgene=fam_vgene[fam].astype(np.int32),
        subgroup=fam_rare[fam].astype(np.int8),
        rep_offsets=np.asarray(rep_offsets, dtype=np.int64),
        params=dict(params, k=3, hash_seed=HASH_SEED, H=GATE_HIDDEN),
    )


def small5k(n_families: int = 500, fam_size: int = 10) -> Repertoire:
    p = WORKLOADS["small5k"]
    rng = np.random.Generator(np.random.PCG64(p["seed"]))
    sizes = np.full(n_families, fam_size)
    codes, lens, fam = families_to_repertoire(rng, sizes, p["Lmin"], p["Lmax"], p["kmax"], p["p_indel"])
    vg = _vgenes_for_families(rng, n_families)
    rare = np.zeros(n_families, dtype=np.int8)
    rare[rng.choice(n_families, max(1, n_families // 100), replace=False)] = 1
    return _finish("small5k", codes, lens, fam, vg, rare, [0, codes.shape[0]], p)


def zipf100k(n: int = 100_000, n_families: int = 10_000) -> Repertoire:
    p = WORKLOADS["zipf100k"]
    rng = np.random.Generator(np.random.PCG64(p["seed"]))
    sizes = zipf_rank_sizes(n, n_families)
    codes, lens, fam = families_to_repertoire(rng, sizes, p["Lmin"], p["Lmax"], p["kmax"], p["p_indel"])
    vg = _vgenes_for_families(rng, n_families)
    rare = np.zeros(n_families, dtype=np.int8)
    rare[rng.choice(n_families, max(1, n_families // 100), replace=False)] = 1
    return _finish("zipf100k", codes, lens, fam, vg, rare, [0, n], p)


def rep1m(n: int = 1_000_000, n_families: int = 100_000, n_rare: int = 2_000) -> Repertoire:
    p = WORKLOADS["rep1m"]
    rng = np.random.Generator(np.random.PCG64(p["seed"]))
    rare_sizes = rng.integers(1, 4, n_rare)
    rest = n - int(rare_sizes.sum())
    m = n_families - n_rare
    common = np.full(m, rest // m, dtype=np.int64)
    common[: rest - int(common.sum())] += 1
    sizes = np.concatenate([common, rare_sizes])
    codes, lens, fam = families_to_repertoire(rng, sizes, p["Lmin"], p["Lmax"], p["kmax"], p["p_indel"])
    vg = _vgenes_for_families(rng, n_families)
    rare = np.zeros(n_families, dtype=np.int8)
    rare[m:] = 1
    return _finish("rep1m", codes, lens, fam, vg, rare, [0, n], p)


def batch_sizes(R: int = 64, lo: float = 1e4, ratio: float = 200.0) -> np.ndarray:
    """Deterministic log-uniform quantiles: n_r = lo * ratio^((r + 1/2) / R)."""
    return np.floor(lo * ratio ** ((np.arange(R) + 0.5) / R)).astype(np.int64)


def batch64(R: int = 64, scale: float = 1.0) -> Repertoire:
    """Many repertoires of uneven size; ``scale`` shrinks every size (for tests)."""
    p = WORKLOADS["batch64"]
    master = np.random.Generator(np.random.PCG64(p["seed"]))
    rep_seeds = master.integers(0, 2**63 - 1, R)
    sizes_r = np.maximum(4, np.floor(batch_sizes(R) * scale).astype(np.int64))
    fam_probs = _zipf_probs(1000)
    parts, fam_base = [], 0
    codes_l, lens_l, fam_l, vg_l, rare_l = [], [], [], [], []
    for r in range(R):
        rng = np.random.Generator(np.random.PCG64(int(rep_seeds[r])))
        nr = int(sizes_r[r])
        est = int(nr / 20) + 16
        fs = []
        tot = 0
        while tot < nr:
            draw = rng.choice(1000, size=est, p=fam_probs) + 1
            for s in draw:
                s = int(min(s, nr - tot))
                fs.append(s)
                tot += s
                if tot >= nr:
                    break
        fs = np.asarray(fs, dtype=np.int64)
        c, l, f = families_to_repertoire(rng, fs, p["Lmin"], p["Lmax"], p["kmax"], p["p_indel"])
        F = fs.shape[0]
        vg = _vgenes_for_families(rng, F)
        rare = np.zeros(F, dtype=np.int8)
        rare[rng.choice(F, max(1, F // 100), replace=False)] = 1
        codes_l.append(c)
        lens_l.append(l)
        fam_l.append(f + fam_base)
        vg_l.append(vg)
        rare_l.append(rare)
        fam_base += F
        parts.append(nr)
    codes = np.concatenate(codes_l)
    lens = np.concatenate(lens_l)
    fam = np.concatenate(fam_l)
    vg = np.concatenate(vg_l)
    rare = np.concatenate(rare_l)
    offs = np.concatenate([[0], np.cumsum(parts)])
    return _finish("batch64", codes, lens, fam, vg, rare, offs, dict(p, R=R, scale=scale))


def tiny(n_families: int = 40, fam_size: int = 6, seed: int = 7, Lmin: int = 8, Lmax: int = 20,
         kmax: int = 3, p_indel: float = 0.1, M: int = 64, b: int = 16, r: int = 4, d: int = 64,
         stride: int = 32) -> Repertoire:
    """Small repertoire for unit tests (any seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.full(n_families, fam_size)
    codes, lens, fam = families_to_repertoire(rng, sizes, Lmin, Lmax, kmax, p_indel, stride)
    vg = _vgenes_for_families(rng, n_families)
    rare = np.zeros(n_families, dtype=np.int8)
    params = dict(seed=seed, Lmin=Lmin, Lmax=Lmax, kmax=kmax, p_indel=p_indel, M=M, b=b, r=r, d=d)
    return _finish("tiny", codes, lens, fam, vg, rare, [0, codes.shape[0]], params)


def concat(reps, name="concat") -> Repertoire:
    """Concatenate repertoires into one batch (family ids made globally unique)."""
    offs = [0]
    fams, base = [], 0
    for rp in reps:
        fams.append(rp.family + base)
        base += int(rp.family.max()) + 1
        offs.append(offs[-1] + rp.n)
    stride = max(rp.stride for rp in reps)
    seqs = np.full((offs[-1], stride), PAD, dtype=np.uint8)
    for rp, o in zip(reps, offs[:-1]):
        seqs[o:o + rp.n, : rp.stride] = rp.seqs
    return Repertoire(
        name=name, seqs=seqs, lens=np.concatenate([rp.lens for rp in reps]),
        family=np.concatenate(fams).astype(np.int32),
        vgene=np.concatenate([rp.vgene for rp in reps]),
        subgroup=np.concatenate([rp.subgroup for rp in reps]),
        rep_offsets=np.asarray(offs, dtype=np.int64), params=dict(reps[0].params))
