"""Shared helpers for the GPU parity tests (inputs come from ``synth``, expected values
from ``oracle``; the GPU path is reached only through the C ABI binding)."""
from __future__ import annotations

import functools
import sys

import numpy as np
import torch

import synth
from oracle import gate as ogate
from oracle import lsh as olsh
from oracle import minhash as omh
from oracle import sw as osw


def say(msg: str) -> None:
    """Name the case before a GPU step (so a failing run says what it was doing)."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(x) -> torch.Tensor:
    if isinstance(x, np.ndarray) and x.dtype == np.uint64:
        x = x.view(np.int64)
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


@functools.lru_cache(maxsize=None)
def workload(name: str):
    return getattr(synth, name)()


@functools.lru_cache(maxsize=None)
def oracle_sig(name: str) -> np.ndarray:
    r = workload(name)
    return omh.signatures_c(r.seqs, r.lens, r.params["M"], synth.HASH_SEED)


@functools.lru_cache(maxsize=None)
def oracle_candidates(name: str) -> np.ndarray:
    """The oracle's whole candidate set of a workload (int64 [P][2], sorted by (i, j))."""
    r = workload(name)
    p = r.params
    offs = r.rep_offsets if len(r.rep_offsets) > 2 else None
    return olsh.candidates_grouped(oracle_sig(name), p["b"], p["r"], rep_offsets=offs)


@functools.lru_cache(maxsize=None)
def oracle_scores(name: str) -> np.ndarray:
    """The C oracle's Smith-Waterman score of every oracle candidate pair of a workload."""
    r = workload(name)
    return osw.scores_pairs(r.seqs, r.lens, oracle_candidates(name), synth.load_blosum62())


def fused_tol_ok(got, ref, rel=1e-5, abs_=1e-6):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    return bool((err <= rel * np.abs(ref) + abs_).all()), float(err.max()) if err.size else 0.0


def grad_tol_ok(got, ref, rel=1e-5, floor=1e-6):
    """Normwise ||d|| <= rel ||ref|| and per element |d| <= rel |ref| + floor * max|ref|."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    d = got - ref
    nref = np.linalg.norm(ref)
    mref = np.abs(ref).max() if ref.size else 0.0
    norm_ok = np.linalg.norm(d) <= rel * nref + 1e-30
    elem_ok = (np.abs(d) <= rel * np.abs(ref) + floor * mref + 1e-30).all()
    return bool(norm_ok and elem_ok), float(np.linalg.norm(d) / max(nref, 1e-300))


def row_candidates_sampled(sig: np.ndarray, rows: np.ndarray, b: int, r: int) -> dict:
    """Oracle candidates of each sampled row (vectorised over all other rows)."""
    return {int(i): olsh.candidates_of_row(sig, int(i), b, r) for i in rows}


def pairs_valid(sig: np.ndarray, pairs: np.ndarray, b: int, r: int) -> bool:
    """Every pair i < j shares at least one band tuple exactly."""
    ok = True
    for lo in range(0, pairs.shape[0], 1 << 20):
        p = pairs[lo:lo + (1 << 20)].astype(np.int64)
        A = sig[p[:, 0], : b * r].reshape(-1, b, r)
        B = sig[p[:, 1], : b * r].reshape(-1, b, r)
        ok &= bool((A == B).all(axis=2).any(axis=1).all())
    return ok and bool((pairs[:, 0] < pairs[:, 1]).all())


def sw_oracle(seqs, lens, pairs, subst, go=10, ge=1):
    return osw.scores_pairs(seqs, lens, pairs, subst, go, ge)


def gate_backward_chunked(oa: dict, grad_f: np.ndarray, chunk: int = 1 << 19) -> dict:
    """The oracle's gate backward over chunks of pairs, summed (the gradient is a sum over
    pairs), so that its per-pair temporaries stay small at millions of pairs."""
    P = oa["pairs"].shape[0]
    out = None
    for lo in range(0, max(P, 1), chunk):
        sl = slice(lo, lo + chunk)
        g = ogate.backward(**dict(oa, pairs=oa["pairs"][sl], align=oa["align"][sl]), grad_f=grad_f[sl])
        if out is None:
            out = g
        else:
            for k in ("W1", "b1", "w2", "b2", "emb"):
                out[k] += g[k]
            out["f"] = np.concatenate([out["f"], g["f"]])
    return out


def ambiguous_flip_bounds(oa: dict, grad_f: np.ndarray, kappa: float = 1e-6):
    """For every hidden unit whose pre-activation lies within float32 rounding of zero (either
    ReLU decision is a correct float32 evaluation), the exact change of each gradient if that
    one decision is flipped.  Returns (number of such units, {name: sum of |change|
    elementwise}, {name: sum of ||change||}): a kernel result that took any mix of those
    decisions lies within these sums of the oracle's own decisions."""
    P = oa["pairs"].shape[0]
    names = ("W1", "b1", "w2", "b2", "emb")
    shapes = {"W1": np.shape(oa["W1"]), "b1": np.shape(oa["b1"]), "w2": np.shape(oa["w2"]),
              "b2": (1,), "emb": np.shape(oa["emb"])}
    elem = {k: np.zeros(shapes[k]) for k in names}
    norm = {k: 0.0 for k in names}
    cells = []
    for lo in range(0, max(P, 1), 1 << 19):
        sl = slice(lo, lo + (1 << 19))
        amb = ogate.relu_ambiguous(**dict(oa, pairs=oa["pairs"][sl], align=oa["align"][sl]), kappa=kappa)
        cells += [(lo + int(p), int(k)) for p, k in zip(*np.nonzero(amb))]
    for p, k in cells:
        pr = oa["pairs"][p:p + 1]
        rows, inv = np.unique(pr.ravel(), return_inverse=True)
        one = dict(oa, emb=oa["emb"][rows], lens=np.asarray(oa["lens"])[rows], vgene=np.asarray(oa["vgene"])[rows],
                   self_scores=np.asarray(oa["self_scores"])[rows], pairs=inv.reshape(1, 2).astype(np.int64),
                   align=oa["align"][p:p + 1])
        _, inter = ogate.forward(**one, return_all=True)
        mask = inter["z"] > 0
        flip = mask.copy()
        flip[0, k] = ~flip[0, k]
        a = ogate.backward(**one, grad_f=grad_f[p:p + 1], relu_mask=mask)
        b = ogate.backward(**one, grad_f=grad_f[p:p + 1], relu_mask=flip)
        for nm in names:
            d = np.abs(b[nm] - a[nm])
            if nm == "emb":
                elem[nm][rows] += d
            else:
                elem[nm] += d.reshape(shapes[nm])
            norm[nm] += float(np.linalg.norm(d))
    return len(cells), elem, norm


def grads_ok_widened(got, ref, elem_w, norm_w, rel=1e-5, floor=1e-6):
    """grad_tol_ok with the bounds widened by the ambiguous-decision sums of
    ambiguous_flip_bounds (zero when no decision is ambiguous)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    ew = np.asarray(elem_w, dtype=np.float64).ravel()
    d = got - ref
    nref = np.linalg.norm(ref)
    mref = np.abs(ref).max() if ref.size else 0.0
    norm_ok = np.linalg.norm(d) <= rel * nref + norm_w + 1e-30
    elem_ok = (np.abs(d) <= rel * np.abs(ref) + floor * mref + ew + 1e-30).all()
    return bool(norm_ok and elem_ok), float(np.linalg.norm(d) / max(nref, 1e-300))
