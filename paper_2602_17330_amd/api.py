"""Python binding of libsubquad: torch tensors in, torch tensors out.

Argument marshalling only -- every step runs in the HIP kernels of libsubquad.so; PyTorch
provides device memory and the current stream. Signatures are returned as int64 tensors
holding the uint64 bit patterns.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import ERR_CAPACITY, SubquadError, check, lib

HASH_SEED = 260217330


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def to_device(x, device="cuda") -> torch.Tensor:
    """numpy / tensor -> contiguous device tensor (uint8/int32/int64/float32 preserved)."""
    if isinstance(x, np.ndarray):
        if x.dtype == np.uint64:
            x = x.view(np.int64)
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device).contiguous()


def check_seqs(seqs: torch.Tensor, lens: torch.Tensor, k: int = 3) -> int:
    """Number of invalid rows; raises SubquadError for bad lengths or residues."""
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    bad = ctypes.c_int64(0)
    check(lib().subquad_check_seqs(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], k,
                                   ctypes.byref(bad), _stream()))
    return bad.value


def minhash(seqs: torch.Tensor, lens: torch.Tensor, M: int, seed: int = HASH_SEED, k: int = 3,
            out: torch.Tensor | None = None) -> torch.Tensor:
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    n = seqs.shape[0]
    if out is None:
        out = torch.empty((n, M), dtype=torch.int64, device=seqs.device)
    check(lib().subquad_minhash(_ptr(seqs), _ptr(lens), n, seqs.shape[1], k, M, seed & (2**64 - 1),
                                _ptr(out), _stream()))
    return out


def lsh_workspace_bytes(n: int, b: int, cap: int) -> int:
    return int(lib().subquad_lsh_workspace_bytes(n, b, cap))


def lsh_candidates(sig: torch.Tensor, b: int, r: int, rep_offsets: torch.Tensor | None = None,
                   cap: int | None = None, with_rows: bool = True):
    """Candidate pairs int32 [P, 2] sorted by (i, j), and CSR row offsets int64 [n + 1]."""
    sig = _dev(sig, torch.int64, "sig")
    n, M = sig.shape
    R = 1
    offs = None
    if rep_offsets is not None:
        offs = _dev(rep_offsets, torch.int64, "rep_offsets")
        R = offs.shape[0] - 1
    cap = int(cap if cap is not None else max(1024, 8 * n))
    dev = sig.device
    rows = torch.empty(n + 1, dtype=torch.int64, device=dev) if with_rows else None
    for _ in range(2):
        ws_bytes = lsh_workspace_bytes(n, b, cap)
        ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
        pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
        P = ctypes.c_int64(0)
        st = lib().subquad_lsh_candidates(_ptr(sig), n, M, b, r, _ptr(offs), R, _ptr(ws), ws_bytes,
                                          _ptr(pairs), _ptr(rows), cap, ctypes.byref(P), _stream())
        if st == ERR_CAPACITY:
            cap = int(P.value)
            continue
        check(st)
        return pairs[: P.value], rows
    raise SubquadError(ERR_CAPACITY, "capacity retry failed")


def self_scores(seqs: torch.Tensor, lens: torch.Tensor, subst: torch.Tensor) -> torch.Tensor:
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    subst = _dev(subst, torch.int8, "subst")
    out = torch.empty(seqs.shape[0], dtype=torch.int32, device=seqs.device)
    check(lib().subquad_self_scores(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], _ptr(subst),
                                    _ptr(out), _stream()))
    return out


def check_subst(subst) -> None:
    """The alignment kernels take a 20x20 matrix in residue-code order (host-side check)."""
    S = subst.detach().cpu().numpy() if isinstance(subst, torch.Tensor) else np.asarray(subst)
    if S.shape != (20, 20):
        raise ValueError("the substitution matrix must be 20x20")


def align_workspace_bytes(P: int) -> int:
    return int(lib().subquad_align_workspace_bytes(P))


def align(seqs: torch.Tensor, lens: torch.Tensor, pairs: torch.Tensor, subst: torch.Tensor,
          gap_open: int = 10, gap_extend: int = 1, out: torch.Tensor | None = None,
          ws: torch.Tensor | None = None) -> torch.Tensor:
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    pairs = _dev(pairs, torch.int32, "pairs")
    subst = _dev(subst, torch.int8, "subst")
    P = pairs.shape[0]
    if out is None:
        out = torch.empty(P, dtype=torch.int32, device=seqs.device)
    if P == 0:
        return out
    need = align_workspace_bytes(P)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=seqs.device)
    check(lib().subquad_align_batch_ws(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1],
                                       _ptr(pairs), P, _ptr(subst), gap_open, gap_extend, _ptr(out),
                                       _ptr(ws), ws.numel(), _stream()))
    return out


def align_dev(seqs, lens, pairs, subst, n_pairs_dev, gap_open=10, gap_extend=1, out=None, ws=None) -> torch.Tensor:
    """Scores of the first ``*n_pairs_dev`` rows of ``pairs`` (a device count; ``pairs`` has the
    capacity's rows).  No host synchronisation."""
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    pairs = _dev(pairs, torch.int32, "pairs")
    subst = _dev(subst, torch.int8, "subst")
    n_pairs_dev = _dev(n_pairs_dev, torch.int64, "n_pairs_dev")
    cap = pairs.shape[0]
    if out is None:
        out = torch.empty(cap, dtype=torch.int32, device=seqs.device)
    need = align_workspace_bytes(cap)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=seqs.device)
    check(lib().subquad_align_batch_dev(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], _ptr(pairs), cap,
                                        _ptr(n_pairs_dev), _ptr(subst), gap_open, gap_extend, _ptr(out), _ptr(ws),
                                        ws.numel(), _stream()))
    return out


def align_noalloc(seqs, lens, pairs, subst, gap_open=10, gap_extend=1, out=None) -> torch.Tensor:
    """The allocation-free entry point (scratch in the library's fixed device array; at most
    ALIGN_NOALLOC_MAX_PAIRS pairs)."""
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    pairs = _dev(pairs, torch.int32, "pairs")
    subst = _dev(subst, torch.int8, "subst")
    if out is None:
        out = torch.empty(pairs.shape[0], dtype=torch.int32, device=seqs.device)
    check(lib().subquad_align_batch_noalloc(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], _ptr(pairs),
                                            pairs.shape[0], _ptr(subst), gap_open, gap_extend, _ptr(out),
                                            _stream()))
    return out


ALIGN_NOALLOC_MAX_PAIRS = 1 << 20


def align_nows(seqs, lens, pairs, subst, gap_open=10, gap_extend=1) -> torch.Tensor:
    """The entry point without a workspace (no length sort)."""
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    pairs = _dev(pairs, torch.int32, "pairs")
    subst = _dev(subst, torch.int8, "subst")
    out = torch.empty(pairs.shape[0], dtype=torch.int32, device=seqs.device)
    check(lib().subquad_align_batch(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], _ptr(pairs),
                                    pairs.shape[0], _ptr(subst), gap_open, gap_extend, _ptr(out),
                                    _stream()))
    return out


def _gate_args(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2):
    emb = _dev(emb, torch.float32, "emb")
    lens = _dev(lens, torch.int32, "lens")
    vgene = _dev(vgene, torch.int32, "vgene")
    self_s = _dev(self_s, torch.int32, "self")
    pairs = _dev(pairs, torch.int32, "pairs")
    align_s = _dev(align_s, torch.int32, "align")
    W1 = _dev(W1, torch.float32, "W1")
    b1 = _dev(b1, torch.float32, "b1")
    w2 = _dev(w2, torch.float32, "w2")
    b2 = _dev(b2, torch.float32, "b2")
    return emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2


def gate_fwd(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2, return_gate: bool = False,
             out: torch.Tensor | None = None):
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2 = _gate_args(
        emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2)
    P = pairs.shape[0]
    fused = out if out is not None else torch.empty(P, dtype=torch.float32, device=emb.device)
    gate = torch.empty(P, dtype=torch.float32, device=emb.device) if return_gate else None
    check(lib().subquad_gate_fwd(_ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene),
                                 _ptr(self_s), _ptr(pairs), _ptr(align_s), P, _ptr(W1), _ptr(b1),
                                 _ptr(w2), _ptr(b2), W1.shape[0], _ptr(fused), _ptr(gate), _stream()))
    return (fused, gate) if return_gate else fused


def gate_bwd_workspace_bytes(H: int, P: int, n: int) -> int:
    need = int(lib().subquad_gate_bwd_workspace_bytes(int(H), int(P), int(n)))
    if need == 0:
        raise SubquadError(1, f"no gate workspace size for H={H}, P={P}, n={n}")
    return need


def gate_bwd(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2, grad_fused,
             need_emb: bool = True, grads=None, ws: torch.Tensor | None = None):
    """Returns (dW1, db1, dw2, db2, demb); accumulates into ``grads`` when given."""
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2 = _gate_args(
        emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2)
    gf = _dev(grad_fused, torch.float32, "grad_fused")
    H = W1.shape[0]
    if grads is None:
        grads = (torch.zeros_like(W1), torch.zeros_like(b1), torch.zeros_like(w2), torch.zeros_like(b2),
                 torch.zeros_like(emb) if need_emb else None)
    dW1, db1, dw2, db2, demb = grads
    need = gate_bwd_workspace_bytes(H, pairs.shape[0], emb.shape[0])
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=emb.device)
    check(lib().subquad_gate_bwd(_ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene),
                                 _ptr(self_s), _ptr(pairs), _ptr(align_s), pairs.shape[0], _ptr(W1),
                                 _ptr(b1), _ptr(w2), _ptr(b2), H, _ptr(gf), _ptr(dW1), _ptr(db1),
                                 _ptr(dw2), _ptr(db2), _ptr(demb), _ptr(ws), ws.numel(), _stream()))
    return dW1, db1, dw2, db2, demb


def gate_train(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2, labels, margin: float = 0.5,
               fused=None, loss=None, grads=None, ws: torch.Tensor | None = None, set_demb: bool = False):
    """Fused forward + contrastive loss + backward.  Returns (fused, loss, (dW1, db1, dw2, db2, demb));
    gradients accumulate into ``grads`` when given, except that with ``set_demb`` the
    embedding gradient is written (no zero fill needed)."""
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2 = _gate_args(
        emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2)
    labels = _dev(labels, torch.int32, "labels")
    H, P = W1.shape[0], pairs.shape[0]
    fused = torch.empty(P, dtype=torch.float32, device=emb.device) if fused is None else fused
    loss = torch.empty(1, dtype=torch.float64, device=emb.device) if loss is None else loss
    if grads is None:
        grads = (torch.zeros_like(W1), torch.zeros_like(b1), torch.zeros_like(w2), torch.zeros_like(b2),
                 torch.zeros_like(emb))
    need = gate_bwd_workspace_bytes(H, P, emb.shape[0])
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=emb.device)
    fn = lib().subquad_gate_train_set if set_demb else lib().subquad_gate_train
    check(fn(_ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene), _ptr(self_s), _ptr(pairs),
             _ptr(align_s), P, _ptr(W1), _ptr(b1), _ptr(w2), _ptr(b2), H, _ptr(labels), margin, _ptr(fused),
             _ptr(loss), *[_ptr(g) for g in grads], _ptr(ws), ws.numel(), _stream()))
    return fused, loss, grads


def gate_train_set_dev(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2, labels, n_pairs_dev,
                       margin: float = 0.5, fused=None, loss=None, grads=None, ws: torch.Tensor | None = None):
    """``gate_train`` with the embedding gradient written, on the first ``*n_pairs_dev`` rows of
    ``pairs`` (a device count; ``pairs`` has the capacity's rows).  No host synchronisation."""
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2 = _gate_args(
        emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2)
    labels = _dev(labels, torch.int32, "labels")
    n_pairs_dev = _dev(n_pairs_dev, torch.int64, "n_pairs_dev")
    H, cap = W1.shape[0], pairs.shape[0]
    fused = torch.empty(cap, dtype=torch.float32, device=emb.device) if fused is None else fused
    loss = torch.empty(1, dtype=torch.float64, device=emb.device) if loss is None else loss
    if grads is None:
        grads = (torch.zeros_like(W1), torch.zeros_like(b1), torch.zeros_like(w2), torch.zeros_like(b2),
                 torch.empty_like(emb))
    need = gate_bwd_workspace_bytes(H, cap, emb.shape[0])
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=emb.device)
    check(lib().subquad_gate_train_set_dev(
        _ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene), _ptr(self_s), _ptr(pairs), _ptr(align_s),
        cap, _ptr(n_pairs_dev), _ptr(W1), _ptr(b1), _ptr(w2), _ptr(b2), H, _ptr(labels), margin, _ptr(fused),
        _ptr(loss), *[_ptr(g) for g in grads], _ptr(ws), ws.numel(), _stream()))
    return fused, loss, grads


class GateFn(torch.autograd.Function):
    """Fused affinity with a hand-written backward: gradients reach the embeddings and the
    gate weights; nothing per pair is saved (the backward recomputes it)."""

    @staticmethod
    def forward(ctx, emb, W1, b1, w2, b2, pairs, align_s, self_s, lens, vgene):
        fused = gate_fwd(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2)
        ctx.save_for_backward(emb, W1, b1, w2, b2, pairs, align_s, self_s, lens, vgene)
        return fused

    @staticmethod
    def backward(ctx, grad_fused):
        emb, W1, b1, w2, b2, pairs, align_s, self_s, lens, vgene = ctx.saved_tensors
        dW1, db1, dw2, db2, demb = gate_bwd(emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2,
                                            grad_fused.contiguous(), need_emb=ctx.needs_input_grad[0])
        return demb, dW1, db1, dw2, db2, None, None, None, None, None


CONTRASTIVE_MARGIN = 0.5


def contrastive_grad(fused, pairs, labels, margin: float = CONTRASTIVE_MARGIN, grad=None, loss=None, ws=None):
    """(grad [P] f32, loss [1] f64) of the per-pair margin contrastive loss on same-label pairs."""
    fused = _dev(fused, torch.float32, "fused")
    pairs = _dev(pairs, torch.int32, "pairs")
    labels = _dev(labels, torch.int32, "labels")
    P = pairs.shape[0]
    grad = torch.empty(P, dtype=torch.float32, device=fused.device) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float64, device=fused.device) if loss is None else loss
    need = int(lib().subquad_contrastive_workspace_bytes())
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=fused.device)
    check(lib().subquad_contrastive_grad(_ptr(fused), _ptr(pairs), P, _ptr(labels), labels.shape[0], margin,
                                         _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(), _stream()))
    return grad, loss


def graph_topk(pairs: torch.Tensor, w: torch.Tensor, n: int, tau: float = 0.7, k: int = 0):
    """CSR similarity graph: (row_offsets int64[n+1], cols int32[nnz], vals float32[nnz])."""
    pairs = _dev(pairs, torch.int32, "pairs")
    w = _dev(w, torch.float32, "w")
    P = pairs.shape[0]
    dev = pairs.device
    need = int(lib().subquad_graph_workspace_bytes(n, P))
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    cap = max(1, 2 * P if k == 0 else min(2 * P, n * k))
    rows = torch.empty(n + 1, dtype=torch.int64, device=dev)
    cols = torch.empty(cap, dtype=torch.int32, device=dev)
    vals = torch.empty(cap, dtype=torch.float32, device=dev)
    nnz = ctypes.c_int64(0)
    check(lib().subquad_graph_topk(_ptr(pairs), _ptr(w), P, n, float(tau), int(k), _ptr(ws), need, _ptr(rows),
                                   _ptr(cols), _ptr(vals), cap, ctypes.byref(nnz), _stream()))
    return rows, cols[: nnz.value], vals[: nnz.value]


EDIT_INDEL = 2


RMT_STEPS = 64
RMT_ITERS = 20
RMT_SEED = 2602


def rmt_threshold(row_offsets, cols, vals, n: int, steps: int = RMT_STEPS, iters: int = RMT_ITERS,
                  seed: int = RMT_SEED, ws=None):
    """(tau*, lambda_plus, lambda_max) of the CSR similarity graph (positive affinities, both
    directions); keep the edges with weight >= tau*."""
    row_offsets = _dev(row_offsets, torch.int64, "row_offsets")
    cols = _dev(cols, torch.int32, "cols")
    vals = _dev(vals, torch.float32, "vals")
    need = int(lib().subquad_rmt_workspace_bytes(n, steps))
    if need == 0:
        raise SubquadError(1, f"no rmt workspace size for n={n}, steps={steps}")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=vals.device)
    out = [ctypes.c_double(0.0) for _ in range(3)]
    check(lib().subquad_rmt_threshold(_ptr(row_offsets), _ptr(cols), _ptr(vals), n, vals.shape[0], steps, iters,
                                      seed, *[ctypes.byref(o) for o in out], _ptr(ws), ws.numel(), _stream()))
    return tuple(o.value for o in out)


def rmt_lambda_max(row_offsets, cols, vals, n: int, tau: float = float("inf"), steps: int = RMT_STEPS,
                   seed: int = RMT_SEED, ws=None) -> float:
    """Largest eigenvalue of the matrix of the edges lighter than tau."""
    row_offsets = _dev(row_offsets, torch.int64, "row_offsets")
    cols = _dev(cols, torch.int32, "cols")
    vals = _dev(vals, torch.float32, "vals")
    need = int(lib().subquad_rmt_workspace_bytes(n, steps))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=vals.device)
    out = ctypes.c_double(0.0)
    check(lib().subquad_rmt_lambda_max(_ptr(row_offsets), _ptr(cols), _ptr(vals), n, vals.shape[0], tau, steps,
                                       seed, ctypes.byref(out), _ptr(ws), ws.numel(), _stream()))
    return out.value


def edit_cost_matrix(subst) -> np.ndarray:
    """Doubled substitution costs of the edit-distance channel (subquad_edit_cost_matrix:
    0 for a match, 1 for a substitution with a positive score, 2 otherwise; indels cost 2)."""
    S = np.ascontiguousarray(subst.detach().cpu().numpy() if isinstance(subst, torch.Tensor) else subst, dtype=np.int8)
    if S.shape != (20, 20):
        raise ValueError("the substitution matrix must be 20x20")
    C = np.empty((20, 20), dtype=np.int8)
    check(lib().subquad_edit_cost_matrix(S.ctypes.data, C.ctypes.data))
    return C


def edit_distance(seqs, lens, pairs, cost, indel: int = EDIT_INDEL, out=None, ws=None) -> torch.Tensor:
    seqs = _dev(seqs, torch.uint8, "seqs")
    lens = _dev(lens, torch.int32, "lens")
    pairs = _dev(pairs, torch.int32, "pairs")
    cost = _dev(cost, torch.int8, "cost")
    P = pairs.shape[0]
    if out is None:
        out = torch.empty(P, dtype=torch.int32, device=seqs.device)
    if P == 0:
        return out
    need = align_workspace_bytes(P)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=seqs.device)
    check(lib().subquad_edit_batch_ws(_ptr(seqs), _ptr(lens), seqs.shape[0], seqs.shape[1], _ptr(pairs), P,
                                      _ptr(cost), indel, _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def _gate3_args(emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2):
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, W2, b2 = _gate_args(
        emb, lens, vgene, self_s, pairs, align_s, W1, b1, W2, b2)
    return emb, lens, vgene, self_s, pairs, align_s, _dev(dist, torch.int32, "dist"), W1, b1, W2, b2


def gate3_fwd(emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2, return_weights=False, out=None):
    emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2 = _gate3_args(
        emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2)
    P = pairs.shape[0]
    fused = out if out is not None else torch.empty(P, dtype=torch.float32, device=emb.device)
    wts = torch.empty((P, 3), dtype=torch.float32, device=emb.device) if return_weights else None
    check(lib().subquad_gate3_fwd(_ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene), _ptr(self_s),
                                  _ptr(pairs), _ptr(align_s), _ptr(dist), P, _ptr(W1), _ptr(b1), _ptr(W2), _ptr(b2),
                                  W1.shape[0], _ptr(fused), _ptr(wts), _stream()))
    return (fused, wts) if return_weights else fused


def gate3_bwd(emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2, grad_fused, need_emb=True):
    emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2 = _gate3_args(
        emb, lens, vgene, self_s, pairs, align_s, dist, W1, b1, W2, b2)
    gf = _dev(grad_fused, torch.float32, "grad_fused")
    H = W1.shape[0]
    grads = (torch.zeros_like(W1), torch.zeros_like(b1), torch.zeros_like(W2), torch.zeros_like(b2),
             torch.zeros_like(emb) if need_emb else None)
    need = int(lib().subquad_gate3_bwd_workspace_bytes(H))
    ws = torch.empty(need, dtype=torch.uint8, device=emb.device)
    check(lib().subquad_gate3_bwd(_ptr(emb), emb.shape[0], emb.shape[1], _ptr(lens), _ptr(vgene), _ptr(self_s),
                                  _ptr(pairs), _ptr(align_s), _ptr(dist), pairs.shape[0], _ptr(W1), _ptr(b1),
                                  _ptr(W2), _ptr(b2), H, _ptr(gf), *[_ptr(g) for g in grads], _ptr(ws), need,
                                  _stream()))
    return grads


PROTO_TAU = 0.1


class ProtoLoss:
    """Prototype-contrastive loss over an embedding table (Eq. (pc), Eq. (proto)); the forward
    keeps its workspace for the backward that follows it."""

    def __init__(self, n: int, d: int, C: int, B: int, device="cuda"):
        self.n, self.d, self.C, self.B = n, d, C, B
        need = int(lib().subquad_proto_workspace_bytes(n, d, C, B))
        if need == 0:
            raise SubquadError(1, f"no proto workspace size for n={n}, d={d}, C={C}, B={B}")
        self.ws = torch.empty(need, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    def _check(self, emb, labels, batch):
        emb = _dev(emb, torch.float32, "emb")
        labels = _dev(labels, torch.int32, "labels")
        batch = _dev(batch, torch.int32, "batch")
        if emb.shape != (self.n, self.d) or labels.shape[0] != self.n or batch.shape[0] != self.B:
            raise SubquadError(1, "shapes do not match the ProtoLoss sizes")
        return emb, labels, batch

    def forward(self, emb, labels, batch, tau: float = PROTO_TAU, row_loss: bool = False, protos: bool = False):
        emb, labels, batch = self._check(emb, labels, batch)
        rl = torch.empty(self.B, dtype=torch.float32, device=emb.device) if row_loss else None
        P = torch.empty((self.C, self.d), dtype=torch.float32, device=emb.device) if protos else None
        check(lib().subquad_proto_fwd(_ptr(emb), self.n, self.d, _ptr(labels), self.C, _ptr(batch), self.B, tau,
                                      _ptr(self.loss), _ptr(rl), _ptr(P), _ptr(self.ws), self.ws.numel(), _stream()))
        return self.loss, rl, P

    def backward(self, emb, labels, batch, tau: float = PROTO_TAU, grad_loss=None, through_prototypes=True,
                 demb=None):
        emb, labels, batch = self._check(emb, labels, batch)
        if demb is None:
            demb = torch.zeros_like(emb)
        gl = None if grad_loss is None else _dev(grad_loss, torch.float32, "grad_loss")
        check(lib().subquad_proto_bwd(_ptr(emb), self.n, self.d, _ptr(labels), self.C, _ptr(batch), self.B, tau,
                                      _ptr(gl), int(bool(through_prototypes)), _ptr(demb), _ptr(self.ws),
                                      self.ws.numel(), _stream()))
        return demb
