"""Shared helpers for the GPU parity tests (inputs come from ``synth``, expected values
from ``oracle``; the GPU path is reached only through the C ABI binding)."""
from __future__ import annotations

import functools
import sys

import numpy as np
import torch

import synth
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
