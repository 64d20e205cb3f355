"""The hot path as one object: buffers are allocated once, every stage runs in libsubquad.

    MinHash -> LSH candidates -> self-scores -> Smith-Waterman -> gate (forward, loss, backward)

A ``Pipeline`` owns the device buffers of one batch of repertoires (signatures, LSH and
alignment workspaces, candidate pairs, scores, fused affinities, gradients), so repeated
steps allocate nothing.  ``step`` runs the whole path once and records a HIP event after every
stage when given events.  The gate stage is one fused pass (forward, contrastive loss and
backward: ``subquad_gate_train``) unless ``PathConfig.fused_gate`` is False, which runs the
separate forward, loss and backward entry points instead.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import api
from ._lib import ERR_CAPACITY, check, lib

STAGES = ("minhash", "lsh", "self", "align", "gate")


@dataclass
class PathConfig:
    M: int = 128
    b: int = 32
    r: int = 4
    gap_open: int = 10
    gap_extend: int = 1
    seed: int = api.HASH_SEED
    margin: float = 0.5
    fused_gate: bool = True


class Pipeline:
    def __init__(self, seqs, lens, vgene, family, emb, subst, W1, b1, w2, b2, cfg: PathConfig,
                 rep_offsets=None, cap: int | None = None, device="cuda"):
        td = lambda x: api.to_device(x, device)  # noqa: E731
        self.cfg = cfg
        self.seqs, self.lens = td(seqs), td(lens)
        self.vgene, self.family = td(vgene), td(family)
        self.emb = td(emb)
        api.check_subst(subst)
        self.subst = td(np.asarray(subst, dtype=np.int8))
        self.W = [td(np.asarray(w, np.float32)) for w in (W1, b1, w2, b2)]
        self.offs = td(np.asarray(rep_offsets, np.int64)) if rep_offsets is not None and len(rep_offsets) > 2 else None
        self.R = 1 if self.offs is None else self.offs.shape[0] - 1
        self.n = int(self.seqs.shape[0])
        self.stride = int(self.seqs.shape[1])
        api.check_seqs(self.seqs, self.lens)
        self.sig = torch.empty((self.n, cfg.M), dtype=torch.int64, device=device)
        self.self_s = torch.empty(self.n, dtype=torch.int32, device=device)
        self.rows = torch.empty(self.n + 1, dtype=torch.int64, device=device)
        self.device = device
        self._alloc_pairs(int(cap) if cap else max(1024, 8 * self.n))
        self.P = 0

    def _alloc_pairs(self, cap: int) -> None:
        self.cap = cap
        dev = self.device
        self.lsh_ws_bytes = int(lib().subquad_lsh_workspace_bytes(self.n, self.cfg.b, cap))
        self.lsh_ws = torch.empty(self.lsh_ws_bytes, dtype=torch.uint8, device=dev)
        self.pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        self.scores = torch.empty(cap, dtype=torch.int32, device=dev)
        self.fused = torch.empty(cap, dtype=torch.float32, device=dev)
        self.align_ws = torch.empty(api.align_workspace_bytes(cap), dtype=torch.uint8, device=dev)
        self.gate_ws = torch.empty(api.gate_bwd_workspace_bytes(self.W[0].shape[0], cap, self.n),
                                   dtype=torch.uint8, device=dev)
        self.grads = [torch.zeros_like(w) for w in self.W] + [torch.zeros_like(self.emb)]
        self.grad_fused_buf = torch.empty(cap, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss_ws = torch.empty(int(lib().subquad_contrastive_workspace_bytes()), dtype=torch.uint8, device=dev)

    # ---------------------------------------------------------------- stages
    def minhash(self):
        api.minhash(self.seqs, self.lens, self.cfg.M, seed=self.cfg.seed, out=self.sig)

    def lsh(self):
        P = ctypes.c_int64(0)
        st = lib().subquad_lsh_candidates(
            self.sig.data_ptr(), self.n, self.cfg.M, self.cfg.b, self.cfg.r,
            None if self.offs is None else self.offs.data_ptr(), self.R, self.lsh_ws.data_ptr(),
            self.lsh_ws_bytes, self.pairs.data_ptr(), self.rows.data_ptr(), self.cap, ctypes.byref(P),
            api._stream())
        if st == ERR_CAPACITY:  # grow once to the exact count, then redo the stage
            self._alloc_pairs(int(P.value * 1.05) + 1024)
            return self.lsh()
        check(st)
        self.P = int(P.value)

    def self_scores(self):
        check(lib().subquad_self_scores(self.seqs.data_ptr(), self.lens.data_ptr(), self.n, self.stride,
                                        self.subst.data_ptr(), self.self_s.data_ptr(), api._stream()))

    def align(self):
        if self.P:
            api.align(self.seqs, self.lens, self.pairs[: self.P], self.subst, self.cfg.gap_open,
                      self.cfg.gap_extend, out=self.scores[: self.P], ws=self.align_ws)

    def gate_args(self):
        P = self.P
        return (self.emb, self.lens, self.vgene, self.self_s, self.pairs[:P], self.scores[:P], *self.W)

    def gate_fwd(self):
        if self.P:
            api.gate_fwd(*self.gate_args(), out=self.fused[: self.P])

    def loss_grad(self):
        """Margin contrastive loss on same-family labels (the gate's training signal)."""
        P = self.P
        api.contrastive_grad(self.fused[:P], self.pairs[:P], self.family, self.cfg.margin,
                             grad=self.grad_fused_buf[:P], loss=self.loss, ws=self.loss_ws)
        self.grad_fused = self.grad_fused_buf[:P]

    def gate_bwd(self):
        for g in self.grads:
            g.zero_()
        if self.P:
            api.gate_bwd(*self.gate_args(), self.grad_fused, grads=tuple(self.grads), ws=self.gate_ws)

    def gate(self):
        """Gate forward, training loss and backward (fused, or the three separate calls)."""
        if not self.cfg.fused_gate:
            self.gate_fwd()
            self.loss_grad()
            self.gate_bwd()
            return
        for g in self.grads[:4]:  # the embedding gradient is written by the training pass itself
            g.zero_()
        P = self.P
        if P:
            api.gate_train(*self.gate_args(), self.family, self.cfg.margin, fused=self.fused[:P], loss=self.loss,
                           grads=tuple(self.grads), ws=self.gate_ws, set_demb=True)
        else:
            self.grads[4].zero_()

    def lsh_async(self):
        """Graph-capturable candidate stage: no host synchronisation; the pair sort is sized
        for the current capacity and the count/status land in device memory."""
        if not hasattr(self, "dev_count"):
            self.dev_count = torch.zeros(1, dtype=torch.int64, device=self.device)
            self.dev_status = torch.zeros(1, dtype=torch.int32, device=self.device)
        check(lib().subquad_lsh_candidates_async(
            self.sig.data_ptr(), self.n, self.cfg.M, self.cfg.b, self.cfg.r,
            None if self.offs is None else self.offs.data_ptr(), self.R, self.lsh_ws.data_ptr(),
            self.lsh_ws_bytes, self.pairs.data_ptr(), self.rows.data_ptr(), self.cap,
            self.dev_count.data_ptr(), self.dev_status.data_ptr(), api._stream()))

    def capture(self):
        """Capture one whole step in a HIP graph (after an eager step has fixed P).

        The candidate stage runs in its asynchronous form with the capacity shrunk to the
        known P; later stages use that P.  Replaying on the same inputs reproduces the eager
        step; ``graph_status()`` reports a capacity overflow if the inputs changed."""
        if self.P == 0:
            self.step()
        P = self.P
        if self.cap != P:
            self._alloc_pairs(max(P, 1))
            self.P = P
        self.lsh_async()          # warm the asynchronous path once outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.minhash()
            self.lsh_async()
            self.self_scores()
            self.align()
            self.gate()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def graph_status(self) -> tuple[int, int]:
        """(device count of candidate pairs, status) of the last asynchronous candidate stage."""
        return int(self.dev_count.item()), int(self.dev_status.item())

    def step(self, events=None):
        """One pass of the whole hot path. ``events``: one CUDA event per stage (STAGES) or None."""
        for k, fn in enumerate((self.minhash, self.lsh, self.self_scores, self.align, self.gate)):
            fn()
            if events is not None:
                events[k].record()

    def cells(self) -> int:
        """Sum over candidate pairs of L_i * L_j (dynamic-programming cells)."""
        pr = self.pairs[: self.P].long()
        L = self.lens.long()
        return int((L[pr[:, 0]] * L[pr[:, 1]]).sum().item())
