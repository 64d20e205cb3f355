"""GPU edit-distance channel (bit-exact) and the three-channel gate (float64 oracle
tolerances) -- the M-channel form of Eq. (wm) with the paper's own edit-distance affinity."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, fused_tol_ok, grad_tol_ok, say, sw_oracle, workload
from oracle import edit as oedit
from oracle import gate as ogate
from oracle import sw as osw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    return synth.load_blosum62()


def test_cost_tables_agree(S):
    assert np.array_equal(sq.edit_cost_matrix(S), oedit.cost_matrix(S))


def _edit_gpu(seqs, lens, pairs, C):
    out = sq.edit_distance(dev(seqs), dev(lens), dev(np.asarray(pairs, np.int32)), dev(C))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_edit_all_pairs_first_thousand(S):
    r = workload("small5k")
    C = oedit.cost_matrix(S)
    iu, ju = np.triu_indices(1000, 1)
    pairs = np.stack([iu, ju], 1).astype(np.int32)
    say("edit distance small5k all pairs 1000")
    assert np.array_equal(_edit_gpu(r.seqs, r.lens, pairs, C), oedit.distances_pairs(r.seqs, r.lens, pairs, C))


@pytest.mark.parametrize("indel", [2, 1, 0, 7])
def test_edit_lengths_1_to_64(S, indel):
    rng = np.random.default_rng(indel)
    n, stride = 300, 64
    lens = rng.integers(1, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    pairs = np.stack([rng.integers(0, n, 3000), rng.integers(0, n, 3000)], 1).astype(np.int32)
    C = oedit.cost_matrix(S)
    say(f"edit distance lengths 1-64 indel={indel}")
    out = sq.edit_distance(dev(seqs), dev(lens), dev(pairs), dev(C), indel=indel)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oedit.distances_pairs(seqs, lens, pairs, C, indel))


def test_edit_rep1m_sampled(S):
    r = workload("rep1m")
    C = oedit.cost_matrix(S)
    pairs = synth.random_pairs(r.n, 2_000_000, 12, family=r.family, same_frac=0.6)
    say("edit distance rep1m 2M pairs")
    got = _edit_gpu(r.seqs, r.lens, pairs, C)
    sel = synth.sample_rows(pairs.shape[0], 50_000, 5)
    assert np.array_equal(got[sel], oedit.distances_pairs(r.seqs, r.lens, pairs[sel], C))


def make_case3(rep, d, H, P, seed, S):
    C = oedit.cost_matrix(S)
    emb = synth.embeddings(rep.seqs, rep.lens, d)
    pairs = synth.random_pairs(rep.n, P, seed, family=rep.family)
    align = sw_oracle(rep.seqs, rep.lens, pairs, S)
    dist = oedit.distances_pairs(rep.seqs, rep.lens, pairs, C)
    rng = np.random.default_rng(seed)
    a1, a2 = 1 / np.sqrt(5), 1 / np.sqrt(H)
    return dict(emb=emb, lens=rep.lens, vgene=rep.vgene, self_scores=osw.self_scores(rep.seqs, rep.lens, S),
                pairs=pairs, align=align, dist=dist,
                W1=rng.uniform(-a1, a1, (H, 5)).astype(np.float32), b1=rng.uniform(-a1, a1, H).astype(np.float32),
                W2=rng.uniform(-a2 * 4, a2 * 4, (3, H)).astype(np.float32),
                b2=rng.uniform(-a2, a2, 3).astype(np.float32))


def _oargs(c):
    e = oedit.similarity(c["dist"], c["lens"], c["pairs"])
    return dict(emb=c["emb"], lens=c["lens"], vgene=c["vgene"], self_scores=c["self_scores"], pairs=c["pairs"],
                align=c["align"], edit_sim=e, W1=c["W1"], b1=c["b1"], W2=c["W2"], b2=c["b2"])


def _gargs(c):
    return (dev(c["emb"]), dev(c["lens"]), dev(c["vgene"]), dev(c["self_scores"]), dev(c["pairs"]),
            dev(c["align"]), dev(c["dist"]), dev(c["W1"]), dev(c["b1"]), dev(c["W2"]), dev(c["b2"]))


@pytest.mark.parametrize("d,H", [(64, 64), (128, 32), (100, 16)])
def test_gate3_forward_backward(S, d, H):
    rep = synth.tiny(n_families=60, fam_size=8, seed=d + H)
    full = make_case3(rep, d, H, 3000, 7, S)
    amb = ogate.relu_ambiguous_m(**_oargs(full)).any(axis=1)
    c = dict(full, pairs=full["pairs"][~amb].copy(), align=full["align"][~amb].copy(),
             dist=full["dist"][~amb].copy())
    say(f"gate3 d={d} H={H} (ambiguous pairs set aside: {int(amb.sum())})")
    f, w = sq.gate3_fwd(*_gargs(c), return_weights=True)
    gf = synth.upstream_grad(c["pairs"].shape[0], seed=d)
    grads = sq.gate3_bwd(*_gargs(c), dev(gf))
    torch.cuda.synchronize()
    fr, inter = ogate.forward_m(**_oargs(c), return_all=True)
    ok, err = fused_tol_ok(f.cpu().numpy(), fr)
    assert ok, err
    assert np.allclose(w.cpu().numpy(), inter["w"], rtol=1e-5, atol=1e-6)
    ref = ogate.backward_m(**_oargs(c), grad_f=gf)
    for name, g in zip(("W1", "b1", "W2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)


def test_gate3_zipf100k_2p20(S):
    """2^20 family-heavy pairs of the 100k Zipf repertoire, d=128, H=64."""
    rep = workload("zipf100k")
    full = make_case3(rep, 128, 64, 1 << 20, 1004, S)
    amb = ogate.relu_ambiguous_m(**_oargs(full)).any(axis=1)
    c = dict(full, pairs=full["pairs"][~amb].copy(), align=full["align"][~amb].copy(),
             dist=full["dist"][~amb].copy())
    say(f"gate3 2^20 (ambiguous pairs set aside: {int(amb.sum())})")
    f = sq.gate3_fwd(*_gargs(c))
    gf = synth.upstream_grad(c["pairs"].shape[0], seed=3)
    grads = sq.gate3_bwd(*_gargs(c), dev(gf))
    torch.cuda.synchronize()
    ref = ogate.backward_m(**_oargs(c), grad_f=gf)
    ok, err = fused_tol_ok(f.cpu().numpy(), ref["f"])
    assert ok, err
    for name, g in zip(("W1", "b1", "W2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)
