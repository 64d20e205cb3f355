"""Benchmark of the SubQuad hot path on one MI355X.

A step is one pass of the whole path over one batch: MinHash signatures -> LSH candidate
pairs -> self-scores -> Smith-Waterman on every candidate -> gated fusion forward ->
(contrastive loss gradient) -> gated fusion backward.  The default workload is the
1,000,000-sequence repertoire (lengths 8-20, 100,000 families, M = 128, 32 x 4 bands,
d = 128, H = 64), inputs resident in HBM before timing.

Prints one JSON line.  ``value`` is whole-step throughput in GCUPS: candidate
dynamic-programming cells (sum of L_i * L_j over candidate pairs) per second of the whole
step.  The Smith-Waterman kernel's own GCUPS, the per-stage times, the gated-fusion
forward+backward rate on 2^20 pairs, the dominant kernel's roofline and the CPU oracle's
rate on a bounded sample are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# int32 VALU lane-ops per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# int32 VALU operations of one folded Gotoh cell update: E and F (two max3 with the extend
# and open terms), diagonal + substitution, H = max3, running max, and the two clamps at 0
SW_OPS_PER_CELL = 8
MFMA_F32_PEAK_TFLOPS = 157.3  # dense fp32 matrix-core peak

# Source files whose text defines each kernel: measured HBM traffic (profiles/hbm_traffic.tsv,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs) is reported only while their hash still
# matches the one recorded with the measurement.
KERNEL_SOURCES = {
    "gate_bwd_kernel": ["gate.hip", "gate_util.h"], "gate_fwd_kernel": ["gate.hip", "gate_util.h"],
    "gate_cos_bwd_j_kernel": ["gate_util.h"], "gate_wgrad_kernel": ["gate.hip", "gate_util.h"],
    "lsh_emit_small_kernel": ["lsh.hip"], "lsh_emit_long_kernel": ["lsh.hip"], "lsh_keys_kernel": ["lsh.hip"],
    "lsh_class_small_kernel": ["lsh.hip"], "lsh_class_long_kernel": ["lsh.hip"],
    "lsh_runs_kernel": ["lsh.hip"], "minhash3_kernel": ["minhash.hip"], "align_kernel": ["align.hip"],
    "radix_scatter_kernel": ["radix.hip"], "radix_hist_kernel": ["radix.hip"],
    "proto_fwd_kernel": ["proto.hip"], "proto_bwd_rows_kernel": ["proto.hip"],
    "proto_bwd_protos_kernel": ["proto.hip"],
}


# Per-pair bytes of the gate's first backward pass with no reuse: the forward's two embedding
# rows, pair, score and output (2 d 4 + 16 = 1,040 at d = 128) plus the i-side gradient row
# (d 4 = 512).  Rows of a repeated i are served from registers and caches, so the rate this
# gives can exceed what HBM moved.
EFFECTIVE_BYTES_PER_PAIR = {"gate_bwd_kernel": 2 * 128 * 4 + 16 + 128 * 4}


def kernel_source_sha(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2602_17330_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """(read + written bytes per launch, detail) from profiles/hbm_traffic.tsv, or (None, reason)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.tsv")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None, "no counter measurement for this kernel"
    rows = [ln.split("\t") for ln in open(path).read().splitlines() if ln and not ln.startswith("#")]
    rows = [r for r in rows if r[0] == kernel]
    if len(rows) != 1:
        return None, "no single counter measurement for this kernel"
    if rows[0][4] != kernel_source_sha(kernel):
        return None, "kernel source changed since the counters were taken"
    rd, wr = float(rows[0][2]), float(rows[0][3])
    return rd + wr, {"read_bytes": rd, "write_bytes": wr, "source": "profiles/pipeline_rep1m_hbm_traffic.md"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rep1m", choices=["rep1m", "zipf100k", "small5k", "batch64"])
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="batch64 only: shrink every repertoire (1.0 = 24.03 M sequences)")
    ap.add_argument("--tune", action="store_true", help="autotune launch shapes before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true", help="skip the 2^20-pair gate measurement")
    ap.add_argument("--gate-2p20-only", action="store_true",
                    help="run only the 2^20-pair gate leg and print its JSON (for counter runs)")
    ap.add_argument("--no-proto", action="store_true", help="skip the prototype-loss measurement")
    ap.add_argument("--no-rmt", action="store_true", help="skip the RMT edge-threshold measurement")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 100k-sequence candidate statistics and steady-state GCUPS")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replayed step")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="also run N elementwise copies of 1 GiB (y = x * 1 over 2^28 float32: 1 GiB read, "
                         "1 GiB written) to calibrate the HBM byte counters")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name):
    import synth
    rep = getattr(synth, name)()
    emb = synth.embeddings(rep.seqs, rep.lens, rep.params["d"])
    return rep, emb


def calib_copy(torch, times):
    """`times` launches of an elementwise copy of 2^28 float32 (1 GiB read, 1 GiB written): the
    known-size kernel that scales the FETCH_SIZE and WRITE_SIZE counters to bytes."""
    if not times:
        return
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(times):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


def time_region(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def config2_leg(torch, sq, steps, warmup):
    """The 100,000-sequence Zipf repertoire (lengths 8-25, M = 128, 32 x 4 bands): candidates
    per query (every candidate pair counts for both its sequences) and steady-state
    Smith-Waterman GCUPS on all its candidate pairs, and on the all-pairs block of its first
    20,000 sequences (199,990,000 pairs), kernels alone (length sort included)."""
    import synth
    from paper_2602_17330_amd import api
    rep = synth.zipf100k()
    S = api.to_device(synth.load_blosum62())
    seqs, lens = api.to_device(rep.seqs), api.to_device(rep.lens)
    sig = sq.minhash(seqs, lens, 128)
    pairs, _ = sq.lsh_candidates(sig, 32, 4)
    P = int(pairs.shape[0])
    deg = torch.bincount(pairs.long().reshape(-1), minlength=rep.n).double()
    q = torch.quantile(deg, torch.tensor([0.5, 0.99], dtype=torch.float64, device=deg.device))
    per_query = dict(mean=float(deg.mean()), p50=float(q[0]), p99=float(q[1]), max=float(deg.max()))
    L = lens.long()

    def sw_rate(pr):
        cells = int((L[pr[:, 0].long()] * L[pr[:, 1].long()]).sum().item())
        out = torch.empty(pr.shape[0], dtype=torch.int32, device="cuda")
        ws = torch.empty(api.align_workspace_bytes(pr.shape[0]), dtype=torch.uint8, device="cuda")
        t = time_region(torch, lambda: api.align(seqs, lens, pr, S, out=out, ws=ws), steps, warmup)
        return dict(pairs=int(pr.shape[0]), cells=cells, ms=t * 1e3, gcups=cells / t / 1e9)

    cand = sw_rate(pairs)
    del pairs
    iu = torch.triu_indices(20_000, 20_000, 1, device="cuda").t().to(torch.int32).contiguous()
    block = sw_rate(iu)
    del iu
    torch.cuda.empty_cache()
    return dict(workload="100,000 synthetic CDR3s (10,000 rank-Zipf(1.5) families), lengths 8-25, M=128, 32x4",
                candidates=P, candidates_per_query=per_query, sw_candidates=cand,
                sw_all_pairs_20k=block)


def gate_2p20(torch, sq, steps, warmup):
    """Gate forward+backward on 2^20 pairs drawn from the 100k-sequence Zipf repertoire's
    candidates (seed 1004), sorted by (i, j); d = 128, H = 64."""
    import synth
    from paper_2602_17330_amd import api
    rep = synth.zipf100k()
    emb = synth.embeddings(rep.seqs, rep.lens, 128)
    S = synth.load_blosum62()
    seqs, lens = api.to_device(rep.seqs), api.to_device(rep.lens)
    sig = sq.minhash(seqs, lens, 128)
    pairs, _ = sq.lsh_candidates(sig, 32, 4)
    Pall = pairs.shape[0]
    rng = np.random.Generator(np.random.PCG64(1004))
    pick = np.sort(rng.choice(Pall, size=min(1 << 20, Pall), replace=False))
    pairs = pairs[torch.from_numpy(pick).cuda()].contiguous()
    St = api.to_device(S)
    align = sq.align(seqs, lens, pairs, St)
    self_s = sq.self_scores(seqs, lens, St)
    W = [api.to_device(w) for w in synth.gate_params(64)]
    E = api.to_device(emb)
    vg = api.to_device(rep.vgene)
    fam = api.to_device(rep.family)
    pr = pairs.long()
    y = (fam[pr[:, 0]] == fam[pr[:, 1]]).float()
    args = (E, lens, vg, self_s, pairs, align, *W)
    fused = torch.empty(pairs.shape[0], dtype=torch.float32, device="cuda")
    grads = [torch.zeros_like(w) for w in W] + [torch.zeros_like(E)]
    ws = torch.empty(api.gate_bwd_workspace_bytes(W[0].shape[0], pairs.shape[0], E.shape[0]), dtype=torch.uint8,
                     device="cuda")
    P = pairs.shape[0]

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    fwd_ms, bwd_ms = [], []

    def one(record=False):
        if record:
            ev[0].record()
        sq.gate_fwd(*args, out=fused)
        if record:
            ev[1].record()
        hinge = torch.clamp(fused - 0.5, min=0.0)
        gf = (-2.0 * y * (1 - fused) + 2.0 * (1 - y) * hinge) / P
        for g in grads:
            g.zero_()
        if record:
            ev[2].record()
        sq.gate_bwd(*args, gf, grads=tuple(grads), ws=ws)
        if record:
            ev[3].record()

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one(record=True)
        torch.cuda.synchronize()
        fwd_ms.append(ev[0].elapsed_time(ev[1]))
        bwd_ms.append(ev[2].elapsed_time(ev[3]))
    wall = (time.perf_counter() - t0) / steps
    f_ms, b_ms = float(np.mean(fwd_ms)), float(np.mean(bwd_ms))
    # the fused training pass (forward + loss + backward in one pass over the pairs)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fam32 = fam.to(torch.int32)

    def train():
        for g in grads:
            g.zero_()
        sq.api.gate_train(*args, fam32, 0.5, fused=fused, loss=loss, grads=tuple(grads), ws=ws)

    train_s = time_region(torch, train, steps, warmup)
    return dict(pairs=P, candidates_total=int(Pall), fwd_ms=f_ms, bwd_ms=b_ms,
                pairs_per_s_kernels=P / ((f_ms + b_ms) / 1e3),
                pairs_per_s_step=P / wall, step_ms=wall * 1e3,
                train_ms=train_s * 1e3, train_pairs_per_s=P / train_s,
                workload="2^20 pairs sampled from the candidates of the 100,000-sequence Zipf "
                         "repertoire, d=128, H=64, fp32")


def proto_leg(torch, sq, rep, emb, steps, warmup):
    """Prototype-contrastive loss (Eq. pc, Eq. proto) forward and backward through the
    prototypes over the bench table: n rows, C = its families, a batch of 65,536 rows
    (seed 78), d = 128, tau = 0.1.  Matrix-core work per step: 2BCd (forward logits) +
    4BCd (batch-row backward: logits again, then G P) + 4BCd (prototype backward: logits
    again, then G^T E)."""
    import synth
    from paper_2602_17330_amd import _lib, api
    labels = rep.family.astype(np.int32)
    C = int(labels.max()) + 1
    B = 65536
    batch = synth.sample_rows(rep.n, B, seed=78).astype(np.int32)
    E = api.to_device(emb)
    Y = api.to_device(labels)
    Bt = api.to_device(batch)
    d = emb.shape[1]
    pl = api.ProtoLoss(rep.n, d, C, B)
    demb = torch.zeros_like(E)

    def one():
        pl.forward(E, Y, Bt)
        pl.backward(E, Y, Bt, demb=demb)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kern = _lib.profile_report()
    _lib.profile_enable(False)
    bcd = 2.0 * B * C * d
    flops = {"proto_fwd_kernel": bcd, "proto_bwd_rows_kernel": 2 * bcd, "proto_bwd_protos_kernel": 2 * bcd}
    kernels = {}
    for name, (launches, total_ms) in kern.items():
        avg = total_ms / max(launches, 1)
        e = {"launches_per_step": launches / steps, "avg_launch_ms": avg}
        if name in flops:
            tf = flops[name] / (avg / 1e3) / 1e12
            e.update(bound="mfma", achieved=tf, peak=MFMA_F32_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=tf / MFMA_F32_PEAK_TFLOPS, alg_flops_per_launch=flops[name])
        kernels[name] = e
    total_flops = 5 * bcd
    return dict(workload=f"{rep.n} rows, C={C} classes (families), B={B}, d={d}, tau=0.1, fp32 MFMA",
                step_ms=wall * 1e3, rows_per_s=B / wall, tflops_step=total_flops / wall / 1e12,
                kernels=kernels)


def rmt_leg(torch, sq, pipe):
    """RMT edge threshold (Sec. 3.7) of the bench step's own similarity graph: every positive
    fused affinity of its candidate pairs, both directions; 64 Lanczos steps per largest
    eigenvalue, 20 bisection steps."""
    from paper_2602_17330_amd import _lib, api
    P = pipe.P
    rows, cols, vals = api.graph_topk(pipe.pairs[:P], pipe.fused[:P], pipe.n, tau=0.0, k=0)
    torch.cuda.synchronize()
    api.rmt_threshold(rows, cols, vals, pipe.n, iters=2)  # warm-up
    torch.cuda.synchronize()
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    tau, lp, lmax = api.rmt_threshold(rows, cols, vals, pipe.n)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # The masked product's rate comes from one full 64-step run (the largest eigenvalue of A
    # itself): bisection runs stop early once a Ritz value clears the bulk edge, and their
    # later launches return at once.
    _lib.profile_enable(True)  # (clears the timings)
    api.rmt_lambda_max(rows, cols, vals, pipe.n, tau=float("inf"))
    torch.cuda.synchronize()
    kern = _lib.profile_report()
    _lib.profile_enable(False)
    nnz = int(vals.shape[0])
    n = pipe.n
    launches, total_ms = kern.get("rmt_spmv_kernel", (0, 0.0))
    avg = total_ms / max(launches, 1)
    alg = nnz * 8 + (n + 1) * 8 + n * 8  # (col, value) per entry, row offsets, x read once, y written
    ach = alg / (avg / 1e3) / 1e9 if avg > 0 else None
    kept = int((vals >= tau).sum().item()) // 2
    return dict(workload=f"similarity graph of the bench step: n={n}, {nnz} directed entries, 64 Lanczos steps, "
                         f"20 bisection steps", ms=wall * 1e3, tau=tau, lambda_plus=lp, lambda_max=lmax,
                edges_kept=kept, edges_total=nnz // 2, spmv_launches_full_run=launches, spmv_avg_ms=avg,
                spmv_roofline={"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS if ach else None, "alg_bytes_per_launch": alg})


# Inputs of the CPU-baseline workers: set before the pool forks, so every task carries only
# an index or a slice bound, never the tables.
_CPU: dict = {}


def _cpu_minhash(bounds):
    """Signatures of rows lo..hi, written into the shared output mapping."""
    from oracle import minhash as omh
    lo, hi = bounds
    d = _CPU
    d["sig"][lo:hi] = omh.signatures_c(d["seqs"][lo:hi], d["lens"][lo:hi], d["M"], d["seed"])


def _cpu_lsh_band(beta):
    """Candidate keys lo * n + hi of one band (the oracle's grouping on that band's rows)."""
    from oracle import lsh as olsh
    d = _CPU
    r = d["r"]
    c = olsh.candidates_grouped(np.ascontiguousarray(d["sig"][:, beta * r:(beta + 1) * r]), 1, r)
    return c[:, 0] * d["sig"].shape[0] + c[:, 1]


def _cpu_sw(bounds):
    from oracle import sw as osw
    lo, hi = bounds
    d = _CPU
    return osw.scores_pairs(d["seqs"], d["lens"], d["pairs"][lo:hi], d["S"], d["go"], d["ge"])


def _cpu_gate(bounds):
    """Gate forward + backward of one chunk of pairs on the rows it touches."""
    from oracle import gate as ogate
    lo, hi = bounds
    d = _CPU
    pr = d["pairs"][lo:hi]
    rows, inv = np.unique(pr.ravel(), return_inverse=True)
    loc = inv.reshape(-1, 2)
    g = ogate.backward(d["emb"][rows], d["lens"][rows], d["vgene"][rows], d["self"][rows], loc,
                       d["align"][lo:hi], *d["W"], d["gf"][lo:hi])
    return rows, g["emb"][: rows.shape[0]], [g[k] for k in ("W1", "b1", "w2", "b2")]


def _cpu_worker_init():
    """One BLAS/OpenMP thread per worker process: ``cores`` processes use ``cores`` cores."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _chunks(n, parts):
    edges = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def cpu_baseline(rep, emb, S, pipe, cfg):
    """The oracle, untouched, timed on the host cores over the same workload.

    MinHash (C loop) and LSH (numpy grouping, one task per band, then the union) run on
    every sequence; Smith-Waterman (C) and the gate forward + backward (numpy float64) run
    on seeded samples of the oracle's own candidate pairs, their times scaled linearly to
    the full workload (DP cells, pairs).  Work is split over a fork pool of ``cores``
    processes; a single-process Smith-Waterman run on part of the sample gives the per-core
    rate beside it."""
    import mmap
    import multiprocessing as mp
    import synth
    from oracle import sw as osw
    cores = min(16, len(os.sched_getaffinity(0)))
    n = rep.n
    _CPU.clear()
    _CPU.update(seqs=np.ascontiguousarray(rep.seqs), lens=np.ascontiguousarray(rep.lens, dtype=np.int32),
                M=cfg.M, seed=synth.HASH_SEED, r=cfg.r, S=np.ascontiguousarray(S, dtype=np.int8),
                go=cfg.gap_open, ge=cfg.gap_extend)
    osw.build()
    ctx = mp.get_context("fork")
    stage = {}
    # the signatures land in an anonymous shared mapping that the forked workers write
    sig_map = mmap.mmap(-1, max(1, n * cfg.M * 8))
    _CPU["sig"] = np.frombuffer(sig_map, dtype=np.uint64, count=n * cfg.M).reshape(n, cfg.M)
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        t = time.perf_counter()
        pool.map(_cpu_minhash, _chunks(n, cores * 4))
        stage["minhash"] = time.perf_counter() - t
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        t = time.perf_counter()
        keys = pool.map(_cpu_lsh_band, range(cfg.b))
        allk = np.unique(np.concatenate(keys))
        cand = np.stack([allk // n, allk % n], axis=1).astype(np.int32)
        stage["lsh"] = time.perf_counter() - t
    del keys, allk
    P_oracle = int(cand.shape[0])
    Ps = min(P_oracle, 2_000_000)
    ps = np.ascontiguousarray(cand[np.sort(synth.sample_rows(P_oracle, Ps, 3))])
    L = rep.lens.astype(np.int64)
    cells_s = int((L[ps[:, 0]] * L[ps[:, 1]]).sum())
    _CPU["pairs"] = ps
    # one core, on the first 5% of the sample
    P1 = max(1, Ps // 20)
    cells_1 = int((L[ps[:P1, 0]] * L[ps[:P1, 1]]).sum())
    t = time.perf_counter()
    osw.scores_pairs(rep.seqs, rep.lens, ps[:P1], S, cfg.gap_open, cfg.gap_extend)
    sw_1core = cells_1 / (time.perf_counter() - t) / 1e9     # (the C loop is single-threaded)
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        t = time.perf_counter()
        al = np.concatenate(pool.map(_cpu_sw, _chunks(Ps, cores * 4)))
        t_sw_s = time.perf_counter() - t
    self_s = osw.self_scores(rep.seqs, rep.lens, S)
    Pg = min(Ps, 250_000)
    _CPU.update(emb=emb, vgene=rep.vgene, self=self_s, align=al, W=synth.gate_params(64),
                gf=synth.upstream_grad(Ps), pairs=ps)
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        t = time.perf_counter()
        parts = pool.map(_cpu_gate, _chunks(Pg, cores * 4))
        dW = [sum(p[2][k] for p in parts) for k in range(4)]
        rows = np.unique(np.concatenate([p[0] for p in parts]))
        dE = np.zeros((rows.shape[0], emb.shape[1]))
        for rr, g, _ in parts:       # rows are unique within a chunk
            dE[np.searchsorted(rows, rr)] += g
        t_gate_s = time.perf_counter() - t
    del parts, dE, dW
    _CPU.clear()
    sig_map.close()
    P = pipe.P
    cells = pipe.cells()  # size of the GPU step's workload, used only to scale the sample times
    stage["align"] = t_sw_s * cells / max(cells_s, 1)
    stage["gate"] = t_gate_s * P / Pg
    total = sum(stage.values())
    sw_gcups = cells_s / t_sw_s / 1e9
    return dict(value=cells / total / 1e9, unit="GCUPS", cores=cores, kind="oracle",
                sample=f"MinHash (C) and LSH (numpy, one task per band) on all {n} sequences; Smith-Waterman "
                       f"(C) on {Ps} and the gate fwd+bwd (numpy fp64) on {Pg} of the oracle's own "
                       f"{P_oracle} candidate pairs (seeded sample), their times scaled linearly to the "
                       f"full workload (DP cells, pairs); {cores} fork-pool processes, one thread each",
                stage_s=stage, oracle_candidates=P_oracle,
                rates={"minhash_seqs_per_s": n / stage["minhash"], "lsh_seqs_per_s": n / stage["lsh"],
                       "sw_gcups": sw_gcups, "sw_gcups_1core": sw_1core,
                       "gate_pairs_per_s": Pg / t_gate_s},
                sw_gcups=sw_gcups)


def bench_batch64(a, torch, sq):
    """Many repertoires of uneven size: one launch per stage over a whole batch (eager, and as
    a replayed HIP graph) against separate per-repertoire launch sequences over the same
    data.  Repertoires are packed into batches that fit the free device memory (Eq. (batch),
    linear footprint behind the prefilter); each leg runs batch after batch, so the
    reported times are sums over the planned batches."""
    import synth
    from paper_2602_17330_amd import _lib, autotune
    from paper_2602_17330_amd.batching import bytes_per_sequence, plan_batches
    from paper_2602_17330_amd.pipeline import PathConfig, Pipeline
    t = time.perf_counter()
    rep = synth.batch64(scale=a.batch_scale)
    log(f"generated {rep.n} sequences in {time.perf_counter() - t:.1f} s")
    S = synth.load_blosum62()
    W = synth.gate_params(64)
    cfg = PathConfig(M=128, b=32, r=4)
    offs = rep.rep_offsets
    sizes = np.diff(offs)
    free, total = torch.cuda.mem_get_info()
    # every leg holds one planned batch at a time (inputs, workspaces, outputs)
    plan = plan_batches(sizes, bytes_per_sequence(128, 32, 128, rep.stride, 40.0), free)
    log(f"batch plan against {free / 2**30:.0f} GiB free: {len(plan)} batch(es) of "
        f"{[int(sizes[b].sum()) for b in plan]} sequences")
    t_per = t_big = t_graph = 0.0
    P_tot = cells = 0
    kern_per, kern_big = {}, {}
    tuned = None
    per_stage_ms = np.zeros(5)
    for bi, reps in enumerate(plan):
        lo, hi = int(offs[reps[0]]), int(offs[reps[-1] + 1])
        emb = synth.embeddings(rep.seqs[lo:hi], rep.lens[lo:hi], 128, device="cuda")
        # (i) separate per-repertoire launch sequences
        per = []
        for k in reps:
            a0, a1 = int(offs[k]) - lo, int(offs[k + 1]) - lo
            pp = Pipeline(rep.seqs[lo + a0:lo + a1], rep.lens[lo + a0:lo + a1], rep.vgene[lo + a0:lo + a1],
                          rep.family[lo + a0:lo + a1], emb[a0:a1], S, *W, cfg=cfg)
            pp.step(check_capacity=True)
            pp.fit_capacity(slack=0.01)
            per.append(pp)
        P_per = sum(pp.P for pp in per)
        cells_b = sum(pp.cells() for pp in per)

        def run_per():
            for pp in per:
                pp.step()

        t_per += time_region(torch, run_per, a.steps, a.warmup)
        _lib.profile_enable(True)
        run_per()
        kern_per = _merge_kernels(kern_per, _lib.profile_report())
        _lib.profile_enable(False)
        del per, pp
        torch.cuda.empty_cache()
        # (ii) one launch per stage over all repertoires of the batch
        boffs = offs[reps[0]:reps[-1] + 2] - lo
        big = Pipeline(rep.seqs[lo:hi], rep.lens[lo:hi], rep.vgene[lo:hi], rep.family[lo:hi], emb, S, *W, cfg=cfg,
                       rep_offsets=boffs)
        big.step(check_capacity=True)
        big.fit_capacity(slack=0.01)
        if big.P != P_per:
            raise RuntimeError(f"batched candidates {big.P} != per-repertoire {P_per}")
        if a.tune and bi == 0:
            tuned = autotune.tune(big)
        t_big += time_region(torch, big.step, a.steps, a.warmup)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record()
        big.step(events=ev[1:])
        torch.cuda.synchronize()
        per_stage_ms += np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(5)])
        _lib.profile_enable(True)
        big.step()
        kern_big = _merge_kernels(kern_big, _lib.profile_report())
        _lib.profile_enable(False)
        big.capture()
        t_graph += time_region(torch, big.replay, a.steps, a.warmup)
        status = big.graph_status()
        if status != (P_per, 0):
            raise RuntimeError(f"graph replay produced {status}, expected ({P_per}, 0)")
        P_tot += P_per
        cells += cells_b
        log(f"batch {bi}: {hi - lo} sequences, P={P_per}; per-repertoire {t_per * 1e3:.1f} ms, "
            f"batched {t_big * 1e3:.1f} ms, graph {t_graph * 1e3:.1f} ms (running sums)")
        del big, emb
        torch.cuda.empty_cache()
    out = {
        "metric": "batched vs per-repertoire hot path (64 repertoires)",
        "value": cells / t_graph / 1e9, "unit": "GCUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t_graph * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch64: 64 repertoires, {rep.n} sequences (log-uniform 1e4..2e6 x "
                               f"{a.batch_scale}), lengths 8-30, i.i.d. Zipf(1.5) family sizes in [1, 1000], "
                               f"M=128, 32x4, d=128, H=64; step = MinHash + LSH + Smith-Waterman + gate "
                               f"(forward, contrastive loss and backward)",
                   "n": rep.n, "candidates": int(P_tot), "cells": int(cells), "batches": len(plan)},
        "per_repertoire_ms": t_per * 1e3, "batched_eager_ms": t_big * 1e3, "batched_graph_ms": t_graph * 1e3,
        "batched_stage_ms": {s: float(m) for s, m in zip(("minhash", "lsh", "self", "align", "gate"), per_stage_ms)},
        "speedup_graph_vs_per_repertoire": t_per / t_graph, "speedup_eager_vs_per_repertoire": t_per / t_big,
        # one step of each leg with every main kernel timed (HIP events): (launches, total ms)
        "kernels_per_repertoire": kern_per, "kernels_batched": kern_big,
        "autotune": tuned,
    }
    print(json.dumps(out), flush=True)


def _merge_kernels(acc, rep):
    for k, (c, ms) in rep.items():
        c0, m0 = acc.get(k, (0, 0.0))
        acc[k] = (c0 + c, m0 + ms)
    return acc


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not "
                                   "part of this build", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import paper_2602_17330_amd as sq
    from paper_2602_17330_amd.pipeline import STAGES, PathConfig, Pipeline
    import synth

    sq.lib()  # fails loudly if the library is missing
    if a.gate_2p20_only:
        out = {"gate_2p20": gate_2p20(torch, sq, max(3, a.steps), a.warmup)}
        calib_copy(torch, a.calib_copy)
        print(json.dumps(out), flush=True)
        return
    if a.workload == "batch64":
        return bench_batch64(a, torch, sq)
    log(f"building workload {a.workload}")
    rep, emb = build_workload(a.workload)
    S = synth.load_blosum62()
    p = rep.params
    cfg = PathConfig(M=p["M"], b=p["b"], r=p["r"])
    W = synth.gate_params(64)
    pipe = Pipeline(rep.seqs, rep.lens, rep.vgene, rep.family, emb, S, *W, cfg=cfg,
                    rep_offsets=rep.rep_offsets)
    log("first pass (sizes the candidate buffers)")
    pipe.step(check_capacity=True)
    pipe.fit_capacity(slack=0.01)  # the capacity a serving loop would keep: the count plus 1%
    P = pipe.P
    cells = pipe.cells()
    log(f"P={P} cells={cells}")
    tuned = None
    if a.tune:
        from paper_2602_17330_amd import autotune
        tuned = autotune.tune(pipe)
        log(f"autotuned: {tuned['best']}")

    from paper_2602_17330_amd import _lib
    for _ in range(a.warmup):
        pipe.step()
    torch.cuda.synchronize()
    # launch times of every main kernel over as many steps as the timed region (each launch
    # bracketed by HIP events on its stream): the kernel table, and which kernel dominates
    _lib.profile_enable(True)
    for _ in range(a.steps):
        pipe.step()
    torch.cuda.synchronize()
    kern = _lib.profile_report()
    _lib.profile_enable(False)
    log("kernels: " + ", ".join(f"{k}={v[1] / a.steps:.3f}ms/step({v[0] // a.steps}x)" for k, v in kern.items()))

    n = rep.n
    M, b, r, d = cfg.M, cfg.b, cfg.r, emb.shape[1]
    pr = pipe.pairs[:P].long()
    rows_i = int(torch.unique(pr[:, 0]).numel())  # distinct first indices
    rows_j = int(torch.unique(pr[:, 1]).numel())
    del pr
    recs = n * b
    # algorithmic bytes (or int32 ops) of ONE launch of each kernel
    alg = {
        "minhash3_kernel": ("hbm", n * (rep.stride + 4) + n * M * 8),
        "lsh_keys_kernel": ("hbm", n * b * r * 8 + recs * 8 + recs * 4),
        "sort_records_scatter": ("hbm", 2 * recs * 8),
        "sort_records_hist": ("hbm", recs * 8),
        # short-run emission: every record read once, every pair key written once (the class
        # rows each visited pair reads are counted by the profiles, not here)
        "lsh_emit_small_kernel": ("hbm", recs * 8 + 8 * P),
        "sort_pairs_scatter": ("hbm", 2 * P * 8),
        "sort_pairs_hist": ("hbm", P * 8),
        # the fused gate pass, compulsory bytes: per pair its partner row, records and outputs,
        # per distinct row its own row and its gradient row (rows by i in the first pass, which
        # writes the gradient rows without reading them; rows by j in the second, which adds
        # to them)
        "gate_bwd_kernel": ("hbm", P * (4 * d + 16 + 4 + 8) + rows_i * (4 * d + 16)
                            + P * (16 + 16 + 4) + rows_i * 4 * d),
        "gate_cos_bwd_j_kernel": ("hbm", P * (8 + 16 + 4 + 4 * d) + rows_j * (4 * d + 4 * d)
                                  + rows_j * 4 * d),
        # (the i-order sort has no roofline entry: the candidate pairs arrive in order of i,
        # so its device-side record count is zero and its launches return at once)
        "sort_gate_j_scatter": ("hbm", 2 * P * 8),
        "sort_lengths_scatter": ("hbm", 2 * P * 8),
        "align_kernel": ("alu", cells * SW_OPS_PER_CELL),
    }

    def kernel_entry(name, launches, total_ms):
        avg_ms = total_ms / max(launches, 1)
        entry = {"launches_per_step": launches / a.steps, "avg_launch_ms": avg_ms, "ms_per_step": total_ms / a.steps}
        if name in alg:
            bound, work = alg[name]
            if bound == "hbm":
                ach = work / (avg_ms / 1e3) / 1e9
                entry.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                             alg_bytes_per_launch=work)
            else:
                ach = work / (avg_ms / 1e3) / 1e12
                entry.update(bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="Tops/s", frac=ach / ALU_PEAK_TOPS,
                             alg_ops_per_launch=work, gcups=cells / (avg_ms / 1e3) / 1e9)
        return entry

    kernels = {name: kernel_entry(name, *v) for name, v in kern.items()}
    dominant = max((k for k in kernels if "bound" in kernels[k]), key=lambda k: kernels[k]["ms_per_step"])

    # timed region: whole steps.  HIP events bracket only the dominant kernel's launches, on
    # its stream, so its roofline figure is measured live here while every other launch runs
    # with no events between them (timing every kernel adds about 0.4 ms of gaps to a step)
    _lib.profile_enable(True)
    _lib.profile_only(dominant)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        pipe.step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / a.steps
    live = _lib.profile_report()
    _lib.profile_only(None)
    _lib.profile_enable(False)
    if dominant not in live or live[dominant][0] != kern[dominant][0]:
        raise RuntimeError(f"the timed region recorded {live.get(dominant)} launches of {dominant}")
    kd = kernel_entry(dominant, *live[dominant])
    log(f"step {wall * 1e3:.3f} ms; {dominant} {kd['avg_launch_ms']:.4f} ms per launch")
    # per-stage split of a few more steps (events between stages, for the stage table)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
    per = np.zeros(len(STAGES))
    reps = max(3, min(a.steps, 10))
    for _ in range(reps):
        ev[0].record()
        pipe.step(events=ev[1:])
        torch.cuda.synchronize()
        per += np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(len(STAGES))])
    stage_ms = per / reps
    log("stages " + ", ".join(f"{s}={m:.3f}" for s, m in zip(STAGES, stage_ms)))
    # the same step replayed from one HIP graph (no launch gaps), reported beside the eager step
    graph_ms = None
    if not a.no_graph:
        pipe.capture()
        pipe.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            pipe.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / a.steps * 1e3
        status = pipe.graph_status()
        if status != (P, 0):
            raise RuntimeError(f"graph replay produced {status}, expected ({P}, 0)")
        log(f"graph-replayed step {graph_ms:.3f} ms")
    traffic, traffic_detail = measured_traffic(dominant)
    roof = {"bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"], "unit": kd["unit"],
            "frac": kd["frac"], "traffic": traffic, "traffic_detail": traffic_detail, "kernel": dominant,
            "avg_launch_ms": kd["avg_launch_ms"],
            "alg_bytes_per_launch": kd.get("alg_bytes_per_launch", kd.get("alg_ops_per_launch"))}
    if traffic:  # the bytes the counters saw, at the same launch time
        roof["traffic_gbs"] = traffic / (kd["avg_launch_ms"] / 1e3) / 1e9
        roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
    eff = EFFECTIVE_BYTES_PER_PAIR.get(dominant)
    if eff:  # the per-pair byte model of the gate (every gather counted, none served by a cache)
        ach = eff * P / (kd["avg_launch_ms"] / 1e3) / 1e9
        roof["effective"] = {"bytes_per_pair": eff, "pairs": P, "achieved": ach, "unit": "GB/s",
                             "frac": ach / HBM_PEAK_GBS}
    sw_gcups = kernels.get("align_kernel", {}).get("gcups")

    gate = None if a.no_gate else gate_2p20(torch, sq, max(3, a.steps), a.warmup)
    cfg2 = None if a.no_config2 else config2_leg(torch, sq, max(3, min(a.steps, 5)), 1)
    proto = None if a.no_proto else proto_leg(torch, sq, rep, emb, max(3, min(a.steps, 5)), 1)
    rmt = None if a.no_rmt else rmt_leg(torch, sq, pipe)
    calib_copy(torch, a.calib_copy)
    cpu = None if a.no_cpu_baseline else cpu_baseline(rep, emb, S, pipe, cfg)

    out = {
        "metric": "SW GCUPS on LSH candidates at 1M CDR3s; gated-fusion fwd+bwd pairs/sec",
        "value": cells / wall / 1e9,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {n} synthetic CDR3s, lengths {p['Lmin']}-{p['Lmax']}, "
                               f"M={M}, {b}x{cfg.r} bands, BLOSUM62 gaps 10/1, d={d}, H=64; step = MinHash + "
                               f"LSH + Smith-Waterman + gate (forward, contrastive loss and backward in "
                               f"one fused pass)",
                   "n": n, "candidates": P, "cells": cells, "parallelism": "single GPU"},
        "sw_kernel_gcups": sw_gcups,
        # the alignment stage alone (length sort, pair metadata, Smith-Waterman), from its events
        "align_stage_gcups": cells / (stage_ms[STAGES.index("align")] / 1e3) / 1e9,
        "stage_ms": {s: float(m) for s, m in zip(STAGES, stage_ms)},
        "graph_ms_per_step": graph_ms,
        "graph_value": cells / (graph_ms / 1e3) / 1e9 if graph_ms else None,
        "gate_2p20": gate,
        "zipf100k": cfg2,
        "proto_loss": proto,
        "rmt_threshold": rmt,
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "autotune": tuned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
