"""The whole hot path end to end (MinHash -> LSH -> Smith-Waterman -> gate forward and
backward) against the oracle chain, batching over repertoires, and determinism."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import (ambiguous_flip_bounds, dev, fused_tol_ok, gate_backward_chunked, grad_tol_ok, grads_ok_widened,
                     host_u64, oracle_candidates, oracle_scores, oracle_sig, say, sw_oracle, workload)
from oracle import gate as ogate
from oracle import lsh as olsh
from oracle import minhash as omh
from oracle import sw as osw

pytestmark = pytest.mark.gpu


def run_gpu(rep, S, emb, W, gf_seed=5):
    p = rep.params
    seqs, lens = dev(rep.seqs), dev(rep.lens)
    offs = dev(rep.rep_offsets) if len(rep.rep_offsets) > 2 else None
    sig = sq.minhash(seqs, lens, p["M"])
    pairs, rows = sq.lsh_candidates(sig, p["b"], p["r"], rep_offsets=offs)
    St = dev(S)
    scores = sq.align(seqs, lens, pairs, St)
    self_s = sq.self_scores(seqs, lens, St)
    args = (dev(emb), lens, dev(rep.vgene), self_s, pairs, scores, *[dev(w) for w in W])
    fused = sq.gate_fwd(*args)
    gf = dev(synth.upstream_grad(pairs.shape[0], seed=gf_seed))
    grads = sq.gate_bwd(*args, gf)
    torch.cuda.synchronize()
    return dict(sig=host_u64(sig), pairs=pairs.cpu().numpy().astype(np.int64), rows=rows.cpu().numpy(),
                scores=scores.cpu().numpy(), fused=fused.cpu().numpy(),
                grads=[g.cpu().numpy() for g in grads])


def test_small5k_end_to_end():
    rep = workload("small5k")
    S = synth.load_blosum62()
    p = rep.params
    emb = synth.embeddings(rep.seqs, rep.lens, p["d"])
    W = synth.gate_params(64)
    say("pipeline small5k")
    got = run_gpu(rep, S, emb, W)
    sig = omh.signatures(rep.seqs, rep.lens, p["M"], synth.HASH_SEED)
    assert np.array_equal(got["sig"], sig)
    pairs = olsh.candidates(sig, p["b"], p["r"])
    assert np.array_equal(got["pairs"], pairs)
    scores = osw.scores_pairs(rep.seqs, rep.lens, pairs, S)
    assert np.array_equal(got["scores"], scores)
    self_s = osw.self_scores(rep.seqs, rep.lens, S)
    oa = dict(emb=emb, lens=rep.lens, vgene=rep.vgene, self_scores=self_s, pairs=pairs, align=scores,
              W1=W[0], b1=W[1], w2=W[2], b2=W[3])
    gf = synth.upstream_grad(pairs.shape[0], seed=5)
    ref = ogate.backward(**oa, grad_f=gf)
    ok, err = fused_tol_ok(got["fused"], ref["f"])
    assert ok, err
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), got["grads"]):
        ok, rel = grad_tol_ok(g, ref[name])
        assert ok, (name, rel)


def test_batched_equals_per_repertoire():
    batch = synth.batch64(R=12, scale=0.004)
    S = synth.load_blosum62()
    emb = synth.embeddings(batch.seqs, batch.lens, 128)
    W = synth.gate_params(64)
    say(f"pipeline batch R=12 n={batch.n}")
    got = run_gpu(batch, S, emb, W)
    offs = batch.rep_offsets
    parts_pairs, parts_scores, parts_fused = [], [], []
    for k in range(len(offs) - 1):
        lo, hi = offs[k], offs[k + 1]
        sub = synth.Repertoire(name="part", seqs=batch.seqs[lo:hi], lens=batch.lens[lo:hi],
                               family=batch.family[lo:hi], vgene=batch.vgene[lo:hi],
                               subgroup=batch.subgroup[lo:hi], rep_offsets=np.array([0, hi - lo]),
                               params=batch.params)
        g = run_gpu(sub, S, emb[lo:hi], W)
        parts_pairs.append(g["pairs"] + lo)
        parts_scores.append(g["scores"])
        parts_fused.append(g["fused"])
    assert np.array_equal(got["pairs"], np.concatenate(parts_pairs))
    assert np.array_equal(got["scores"], np.concatenate(parts_scores))
    assert np.allclose(got["fused"], np.concatenate(parts_fused), rtol=1e-6, atol=1e-7)
    # and against the oracle on the whole batch
    sig = omh.signatures(batch.seqs, batch.lens, 128, synth.HASH_SEED)
    assert np.array_equal(got["sig"], sig)
    assert np.array_equal(got["pairs"], olsh.candidates_grouped(sig, 32, 4, rep_offsets=offs))


def test_two_runs_identical():
    rep = workload("small5k")
    S = synth.load_blosum62()
    emb = synth.embeddings(rep.seqs, rep.lens, 64)
    W = synth.gate_params(64)
    say("pipeline determinism")
    a = run_gpu(rep, S, emb, W)
    b = run_gpu(rep, S, emb, W)
    for k in ("sig", "pairs", "rows", "scores", "fused"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(a["grads"][:4], b["grads"][:4]):
        assert np.array_equal(x, y)
    assert np.allclose(a["grads"][4], b["grads"][4], rtol=1e-5, atol=1e-7)


def test_graph_replay_matches_eager():
    """The whole step captured in a HIP graph; replays (with eager work and host syncs in
    between) reproduce the eager step bit for bit on the integer stages."""
    from paper_2602_17330_amd.pipeline import PathConfig, Pipeline
    rep = workload("small5k")
    S = synth.load_blosum62()
    emb = synth.embeddings(rep.seqs, rep.lens, 64)
    W = synth.gate_params(64)
    say("pipeline graph capture")
    pipe = Pipeline(rep.seqs, rep.lens, rep.vgene, rep.family, emb, S, *W,
                    cfg=PathConfig(M=64, b=16, r=4))
    pipe.step()
    torch.cuda.synchronize()
    P = pipe.P
    eager = dict(sig=pipe.sig.clone(), pairs=pipe.pairs[:P].clone(), scores=pipe.scores[:P].clone(),
                 fused=pipe.fused[:P].clone(), grads=[g.clone() for g in pipe.grads])
    pipe.capture()
    for k in range(3):
        pipe.sig.zero_()
        pipe.scores.zero_()
        pipe.fused.zero_()
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        pipe.replay()
        torch.cuda.synchronize()
        assert pipe.graph_status() == (P, 0)
        assert torch.equal(pipe.sig, eager["sig"])
        assert torch.equal(pipe.pairs[:P], eager["pairs"])
        assert torch.equal(pipe.scores[:P], eager["scores"])
        assert torch.allclose(pipe.fused[:P], eager["fused"], rtol=1e-6, atol=1e-7)
        for a, b in zip(pipe.grads[:4], eager["grads"][:4]):
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-7)
        assert torch.allclose(pipe.grads[4], eager["grads"][4], rtol=1e-4, atol=1e-6)
        del junk


def test_graph_replays_on_a_new_batch():
    """One captured step replayed on new inputs of the same shape (other sequences, other
    repertoire boundaries, another candidate count): the replay equals an eager step on
    those inputs with the same capacity and the oracle; a batch whose candidates overflow
    the capacity is reported by the status, not run past it."""
    from paper_2602_17330_amd.pipeline import PathConfig, Pipeline
    S = synth.load_blosum62()
    W = synth.gate_params(64)
    cfg = PathConfig(M=64, b=16, r=4)

    def batch(parts):
        rep = synth.concat([synth.tiny(n_families=f, fam_size=m, seed=sd) for f, m, sd in parts])
        return rep, synth.embeddings(rep.seqs, rep.lens, 64)

    A, eA = batch([(150, 8, 21), (100, 6, 22)])            # 1200 + 600 sequences
    B, eB = batch([(100, 9, 23), (150, 6, 24)])            # 900 + 900: other boundaries
    assert A.n == B.n
    say(f"pipeline graph on a new batch n={A.n}")
    pipe = Pipeline(A.seqs, A.lens, A.vgene, A.family, eA, S, *W, cfg=cfg, rep_offsets=A.rep_offsets)
    pipe.step(check_capacity=True)
    P_A = pipe.P
    pipe.fit_capacity(slack=1.0)                              # room for a batch with more pairs
    cap = pipe.cap
    pipe.capture()
    pipe.load(seqs=B.seqs, lens=B.lens, vgene=B.vgene, family=B.family, emb=eB, rep_offsets=B.rep_offsets)
    for k in range(2):
        pipe.fused.zero_()
        torch.cuda.synchronize()
        pipe.replay()
        torch.cuda.synchronize()
        P_B, status = pipe.graph_status()
        assert status == 0 and P_B != P_A and P_B <= cap
        ref = Pipeline(B.seqs, B.lens, B.vgene, B.family, eB, S, *W, cfg=cfg, rep_offsets=B.rep_offsets, cap=cap)
        ref.step()
        assert ref.graph_status() == (P_B, 0)
        assert torch.equal(pipe.sig, ref.sig)
        assert torch.equal(pipe.pairs[:P_B], ref.pairs[:P_B])
        assert torch.equal(pipe.scores[:P_B], ref.scores[:P_B])
        assert torch.equal(pipe.fused[:P_B], ref.fused[:P_B])
        for a, b in zip(pipe.grads[:4], ref.grads[:4]):
            assert torch.equal(a, b)
        assert torch.allclose(pipe.grads[4], ref.grads[4], rtol=1e-5, atol=1e-7)
        assert abs(pipe.loss.item() - ref.loss.item()) <= 1e-12 * abs(ref.loss.item())
        del ref
    sig = omh.signatures(B.seqs, B.lens, 64, synth.HASH_SEED)
    pairs = olsh.candidates_grouped(sig, 16, 4, rep_offsets=B.rep_offsets)
    assert np.array_equal(pipe.pairs[:P_B].cpu().numpy().astype(np.int64), pairs)
    assert np.array_equal(pipe.scores[:P_B].cpu().numpy(), osw.scores_pairs(B.seqs, B.lens, pairs, S))
    # a batch with more candidates than the capacity: flagged, with its exact count
    C = synth.concat([synth.tiny(n_families=30, fam_size=40, seed=25), synth.tiny(n_families=30, fam_size=20, seed=26)])
    assert C.n == A.n
    sigC = omh.signatures(C.seqs, C.lens, 64, synth.HASH_SEED)
    P_C = olsh.candidates_grouped(sigC, 16, 4, rep_offsets=C.rep_offsets).shape[0]
    assert P_C > cap
    pipe.load(seqs=C.seqs, lens=C.lens, vgene=C.vgene, family=C.family,
              emb=synth.embeddings(C.seqs, C.lens, 64), rep_offsets=C.rep_offsets)
    say(f"pipeline graph overflow P={P_C} cap={cap}")
    pipe.replay()
    torch.cuda.synchronize()
    assert pipe.graph_status() == (P_C, 4)


def test_knobs_never_change_results():
    """Launch-shape knobs (the autotuner's search space) leave every result unchanged."""
    from paper_2602_17330_amd import autotune
    rep = workload("small5k")
    S = synth.load_blosum62()
    emb = synth.embeddings(rep.seqs, rep.lens, 64)
    W = synth.gate_params(64)
    say("knob invariance")
    base = run_gpu(rep, S, emb, W)
    try:
        for name, vals in autotune.CANDIDATES.items():
            for v in vals:
                autotune.set_knob(name, v)
                got = run_gpu(rep, S, emb, W)
                for k in ("sig", "pairs", "rows", "scores"):
                    assert np.array_equal(got[k], base[k]), (name, v, k)
                assert np.allclose(got["fused"], base["fused"], rtol=1e-6, atol=1e-7)
            autotune.set_knob(name, 0)
    finally:
        autotune.reset()


def test_pipeline_step_against_oracle():
    """Pipeline.step() on small5k (fused gate pass: forward, contrastive loss on same-family
    labels, backward) against the oracle chain.  Its one pair with a ReLU pre-activation within
    float32 rounding of zero is checked against either decision on its ambiguous units."""
    import itertools
    from paper_2602_17330_amd.pipeline import PathConfig, Pipeline
    rep = workload("small5k")
    S = synth.load_blosum62()
    p = rep.params
    emb = synth.embeddings(rep.seqs, rep.lens, p["d"])
    W = synth.gate_params(64)
    say("pipeline step small5k (fused gate)")
    pipe = Pipeline(rep.seqs, rep.lens, rep.vgene, rep.family, emb, S, *W,
                    cfg=PathConfig(M=p["M"], b=p["b"], r=p["r"]))
    pipe.step()
    torch.cuda.synchronize()
    P = pipe.P
    sig = omh.signatures(rep.seqs, rep.lens, p["M"], synth.HASH_SEED)
    pairs = olsh.candidates(sig, p["b"], p["r"])
    assert np.array_equal(pipe.pairs[:P].cpu().numpy(), pairs)
    scores = osw.scores_pairs(rep.seqs, rep.lens, pairs, S)
    assert np.array_equal(pipe.scores[:P].cpu().numpy(), scores)
    oa = dict(emb=emb, lens=rep.lens, vgene=rep.vgene, self_scores=osw.self_scores(rep.seqs, rep.lens, S),
              pairs=pairs, align=scores, W1=W[0], b1=W[1], w2=W[2], b2=W[3])
    f64, inter = ogate.forward(**oa, return_all=True)
    ok, err = fused_tol_ok(pipe.fused[:P].cpu().numpy(), f64)
    assert ok, err
    y = (rep.family[pairs[:, 0]] == rep.family[pairs[:, 1]]).astype(np.float64)
    L, gl = ogate.contrastive_loss(f64, y, 0.5)
    assert abs(pipe.loss.item() - L) <= 1e-5 * L
    got = [g.cpu().numpy() for g in pipe.grads]
    amb = ogate.relu_ambiguous(**oa)
    cells = list(zip(*np.nonzero(amb)))[:6]
    ok_any = False
    for bits in itertools.product([False, True], repeat=len(cells)):
        mask = inter["z"] > 0
        for (pp, k), bit in zip(cells, bits):
            mask[pp, k] = bit
        ref = ogate.backward(**oa, grad_f=gl, relu_mask=mask)
        if all(grad_tol_ok(g, ref[nm])[0] for nm, g in zip(("W1", "b1", "w2", "b2", "emb"), got)):
            ok_any = True
            break
    assert ok_any


def test_pipeline_step_rep1m_against_oracle():
    """The benchmark's own step (Pipeline.step on the 1M-sequence workload, M = 128, 32 x 4,
    d = 128, H = 64, the fused gate pass with the embedding gradient written) against the
    oracle chain at full size: every signature, the whole candidate set, every alignment
    score, every fused value, the loss and every gradient element (bounds widened by the
    ReLU decisions float32 may take either way)."""
    from paper_2602_17330_amd.pipeline import PathConfig, Pipeline
    rep = workload("rep1m")
    S = synth.load_blosum62()
    p = rep.params
    emb = synth.embeddings(rep.seqs, rep.lens, p["d"])
    W = synth.gate_params(64)
    say("pipeline step rep1m")
    pipe = Pipeline(rep.seqs, rep.lens, rep.vgene, rep.family, emb, S, *W,
                    cfg=PathConfig(M=p["M"], b=p["b"], r=p["r"]), rep_offsets=rep.rep_offsets)
    pipe.step()
    pipe.step()                 # a second step over the same buffers (the benchmark repeats steps)
    torch.cuda.synchronize()
    P = pipe.P
    got_sig = host_u64(pipe.sig)
    got_pairs = pipe.pairs[:P].cpu().numpy().astype(np.int64)
    got_scores = pipe.scores[:P].cpu().numpy()
    got_fused = pipe.fused[:P].cpu().numpy()
    got_loss = pipe.loss.item()
    got = [g.cpu().numpy() for g in pipe.grads]
    del pipe
    torch.cuda.empty_cache()
    say(f"pipeline step rep1m: P={P}; oracle signatures and candidates")
    assert np.array_equal(got_sig, oracle_sig("rep1m"))
    del got_sig
    pairs = oracle_candidates("rep1m")
    assert np.array_equal(got_pairs, pairs)
    say("pipeline step rep1m: oracle alignment scores")
    scores = oracle_scores("rep1m")
    assert np.array_equal(got_scores, scores)
    say("pipeline step rep1m: oracle gate forward")
    oa = dict(emb=emb, lens=rep.lens, vgene=rep.vgene, self_scores=osw.self_scores(rep.seqs, rep.lens, S),
              pairs=pairs, align=scores, W1=W[0], b1=W[1], w2=W[2], b2=W[3])
    f64 = np.concatenate([ogate.forward(**dict(oa, pairs=pairs[lo:lo + (1 << 19)], align=scores[lo:lo + (1 << 19)]))
                          for lo in range(0, P, 1 << 19)])
    ok, err = fused_tol_ok(got_fused, f64)
    assert ok, err
    y = (rep.family[pairs[:, 0]] == rep.family[pairs[:, 1]]).astype(np.float64)
    L, gl = ogate.contrastive_loss(f64, y, 0.5)
    assert abs(got_loss - L) <= 1e-5 * abs(L)
    say("pipeline step rep1m: oracle gate backward")
    ref = gate_backward_chunked(oa, gl)
    n_amb, ew, nw = ambiguous_flip_bounds(oa, gl)
    say(f"pipeline step rep1m: {n_amb} ambiguous ReLU decisions")
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), got):
        ok, rel = grads_ok_widened(g, ref[name], ew[name], nw[name])
        assert ok, (name, rel)
