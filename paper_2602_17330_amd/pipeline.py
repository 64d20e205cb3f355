"""The hot path as one object: buffers are allocated once, every stage runs in libsubquad.

    MinHash -> LSH candidates -> self-scores -> Smith-Waterman -> gate (forward, loss, backward)

A ``Pipeline`` owns the device buffers of one batch of repertoires (signatures, LSH and
alignment workspaces, candidate pairs, scores, fused affinities, gradients), so repeated
steps allocate nothing.  ``step`` runs the whole path once and records a HIP event after every
stage when given events; the candidate count never leaves the device inside a step.  The gate stage is one fused pass (forward, contrastive loss and
backward: ``subquad_gate_train``) unless ``PathConfig.fused_gate`` is False, which runs the
separate forward, loss and backward entry points instead.
"""
from __future__ import annotations

import math
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
    """The whole path over one batch, with its buffers allocated once.

    The candidate count P stays on the device: the candidate stage leaves it (and an
    overflow status) in ``dev_count`` / ``dev_status``, and the alignment and fused gate
    stages read it there, with launches sized for the capacity ``cap``.  A step therefore
    never waits on the host, and one captured HIP graph replays on new inputs of the same
    shape (``load``), as long as their P fits ``cap`` (``graph_status``).  ``P`` reads the
    count back (one synchronisation); ``step(check_capacity=True)`` grows the capacity and redoes the
    step when the candidates overflowed it."""

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
        self.dev_count = torch.zeros(1, dtype=torch.int64, device=device)
        self.dev_status = torch.zeros(1, dtype=torch.int32, device=device)
        self.device = device
        self.graph = None
        self._alloc_pairs(int(cap) if cap else max(1024, 8 * self.n))

    def _alloc_pairs(self, cap: int) -> None:
        self.cap = cap
        self.graph = None  # a captured graph holds the old buffers' addresses
        dev = self.device
        for name in ("lsh_ws", "pairs", "scores", "fused", "align_ws", "gate_ws", "grad_fused_buf"):
            self.__dict__.pop(name, None)  # free the old buffers before the new ones are taken
        self.lsh_ws_bytes = int(lib().subquad_lsh_workspace_bytes(self.n, self.cfg.b, cap))
        self.lsh_ws = torch.empty(self.lsh_ws_bytes, dtype=torch.uint8, device=dev)
        self.pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        self.scores = torch.empty(cap, dtype=torch.int32, device=dev)
        self.fused = torch.empty(cap, dtype=torch.float32, device=dev)
        self.align_ws = torch.empty(api.align_workspace_bytes(cap), dtype=torch.uint8, device=dev)
        self.gate_ws = torch.empty(api.gate_bwd_workspace_bytes(self.W[0].shape[0], cap, self.n),
                                   dtype=torch.uint8, device=dev)
        if not hasattr(self, "grads"):
            self.grads = [torch.zeros_like(w) for w in self.W] + [torch.zeros_like(self.emb)]
        self.grad_fused_buf = torch.empty(cap, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss_ws = torch.empty(int(lib().subquad_contrastive_workspace_bytes()), dtype=torch.uint8, device=dev)

    def load(self, seqs=None, lens=None, vgene=None, family=None, emb=None, rep_offsets=None) -> None:
        """Copy a new batch of the same shape (n sequences, stride, R repertoires) into the
        input buffers; a captured graph then runs on it.  Lengths and residue codes are
        validated as in the constructor."""
        if rep_offsets is not None and self.offs is None:
            if len(rep_offsets) != 2:
                raise ValueError("this pipeline was built for one repertoire")
            rep_offsets = None
        for name, x in (("seqs", seqs), ("lens", lens), ("vgene", vgene), ("family", family), ("emb", emb),
                        ("offs", None if rep_offsets is None else np.asarray(rep_offsets, np.int64))):
            if x is None:
                continue
            dst = getattr(self, name)
            src = api.to_device(x, self.device)
            if src.shape != dst.shape or src.dtype != dst.dtype:
                raise ValueError(f"{name}: expected {tuple(dst.shape)} {dst.dtype}, got {tuple(src.shape)} {src.dtype}")
            dst.copy_(src)
        api.check_seqs(self.seqs, self.lens)

    # ---------------------------------------------------------------- stages
    def minhash(self):
        api.minhash(self.seqs, self.lens, self.cfg.M, seed=self.cfg.seed, out=self.sig)

    def lsh(self):
        """Candidate stage: pairs, CSR rows, and the count and status left on the device."""
        check(lib().subquad_lsh_candidates_async(
            self.sig.data_ptr(), self.n, self.cfg.M, self.cfg.b, self.cfg.r,
            None if self.offs is None else self.offs.data_ptr(), self.R, self.lsh_ws.data_ptr(),
            self.lsh_ws_bytes, self.pairs.data_ptr(), self.rows.data_ptr(), self.cap,
            self.dev_count.data_ptr(), self.dev_status.data_ptr(), api._stream()))

    def self_scores(self):
        check(lib().subquad_self_scores(self.seqs.data_ptr(), self.lens.data_ptr(), self.n, self.stride,
                                        self.subst.data_ptr(), self.self_s.data_ptr(), api._stream()))

    def align(self):
        api.align_dev(self.seqs, self.lens, self.pairs, self.subst, self.dev_count, self.cfg.gap_open,
                      self.cfg.gap_extend, out=self.scores, ws=self.align_ws)

    @property
    def P(self) -> int:
        """The candidate count of the last candidate stage (synchronises; raises if it
        overflowed the capacity)."""
        P, status = self.graph_status()
        if status != 0:
            raise RuntimeError(f"{P} candidate pairs overflow the capacity of {self.cap}")
        return P

    def gate_args(self):
        P = self.P
        return (self.emb, self.lens, self.vgene, self.self_s, self.pairs[:P], self.scores[:P], *self.W)

    def gate_fwd(self):
        P = self.P
        if P:
            api.gate_fwd(*self.gate_args(), out=self.fused[:P])

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
        """Gate forward, training loss and backward: one fused pass on the device count (or,
        with ``fused_gate=False``, the three separate calls on the count read back)."""
        if not self.cfg.fused_gate:
            self.gate_fwd()
            self.loss_grad()
            self.gate_bwd()
            return
        for g in self.grads[:4]:  # the embedding gradient is written by the training pass itself
            g.zero_()
        api.gate_train_set_dev(self.emb, self.lens, self.vgene, self.self_s, self.pairs, self.scores, *self.W,
                               self.family, self.dev_count, self.cfg.margin, fused=self.fused, loss=self.loss,
                               grads=tuple(self.grads), ws=self.gate_ws)

    def step(self, events=None, check_capacity: bool = False):
        """One pass of the whole hot path. ``events``: one CUDA event per stage (STAGES) or None.
        ``check_capacity``: read the count back and, if the candidates overflowed the
        capacity, grow it to fit and run the step again."""
        for k, fn in enumerate((self.minhash, self.lsh, self.self_scores, self.align, self.gate)):
            fn()
            if events is not None:
                events[k].record()
        if check_capacity:
            P, status = self.graph_status()
            if status == ERR_CAPACITY:
                self._alloc_pairs(int(P * 1.05) + 1024)
                self.step(events, check_capacity=False)
                assert self.graph_status()[1] == 0

    def fit_capacity(self, slack: float = 0.0) -> None:
        """Resize the pair buffers to the last count plus ``slack`` (a fraction of it).  New
        buffers hold no results yet, so the step is run again on them."""
        P = self.P
        cap = max(1, P + int(math.ceil(P * slack)))
        if cap != self.cap:
            self._alloc_pairs(cap)
            self.step()
            if self.graph_status() != (P, 0):
                raise RuntimeError("the step gave another candidate count on the same inputs")

    def capture(self):
        """Capture one whole step in a HIP graph.  It keeps the current buffers and capacity:
        replays run on whatever ``load`` put in the input buffers."""
        self.step(check_capacity=True)  # warm every path once outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def graph_status(self) -> tuple[int, int]:
        """(device count of candidate pairs, status) of the last candidate stage."""
        return int(self.dev_count.item()), int(self.dev_status.item())

    def cells(self) -> int:
        """Sum over candidate pairs of L_i * L_j (dynamic-programming cells)."""
        pr = self.pairs[: self.P].long()
        L = self.lens.long()
        return int((L[pr[:, 0]] * L[pr[:, 1]]).sum().item())
