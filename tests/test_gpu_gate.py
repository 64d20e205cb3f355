"""GPU gate forward/backward against the float64 oracle.

Tolerances (float32 kernels against float64): fused |f - f64| <= 1e-5 |f64| + 1e-6; gradients
normwise ||d|| <= 1e-5 ||ref|| and per element |d| <= 1e-5 |ref| + 1e-6 max|ref|."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import (ambiguous_flip_bounds, dev, fused_tol_ok, gate_backward_chunked, grad_tol_ok, grads_ok_widened,
                     oracle_candidates, oracle_scores, say, sw_oracle, workload)
from oracle import gate as ogate
from oracle import sw as osw

pytestmark = pytest.mark.gpu


def make_case(rep, d, H, P, seed, same_frac=0.5, scale_norms=False, gseed=77):
    S = synth.load_blosum62()
    emb = synth.embeddings(rep.seqs, rep.lens, d)
    if scale_norms:
        rng = np.random.default_rng(seed)
        emb = (emb * rng.uniform(0.25, 4.0, (rep.n, 1))).astype(np.float32)
    pairs = synth.random_pairs(rep.n, P, seed, family=rep.family, same_frac=same_frac)
    align = sw_oracle(rep.seqs, rep.lens, pairs, S)
    self_s = osw.self_scores(rep.seqs, rep.lens, S)
    W1, b1, w2, b2 = synth.gate_params(H, seed=gseed)
    return dict(emb=emb, lens=rep.lens, vgene=rep.vgene, self_scores=self_s, pairs=pairs, align=align,
                W1=W1, b1=b1, w2=w2, b2=b2, family=rep.family)


def split_ambiguous(c, kappa=1e-6):
    """(case without the pairs whose ReLU decisions are ambiguous at float32 precision,
    indices of those pairs in the original case)."""
    amb = ogate.relu_ambiguous(**oracle_args(c), kappa=kappa).any(axis=1)
    keep = ~amb
    c2 = dict(c, pairs=np.ascontiguousarray(c["pairs"][keep]), align=np.ascontiguousarray(c["align"][keep]))
    return c2, np.nonzero(amb)[0]


def check_ambiguous_pairs(c, idx, gf, kappa=1e-6):
    """Each ambiguous pair alone: the GPU gradient must match the oracle with the kernel's
    ReLU decision taken either way on every ambiguous unit."""
    import itertools
    for p in idx[:16]:
        c1 = dict(c, pairs=np.ascontiguousarray(c["pairs"][p:p + 1]),
                  align=np.ascontiguousarray(c["align"][p:p + 1]))
        g1 = gf[p:p + 1]
        grads = [t.cpu().numpy() for t in sq.gate_bwd(*gpu_args(c1), dev(g1))]
        torch.cuda.synchronize()
        _, inter = ogate.forward(**oracle_args(c1), return_all=True)
        amb = ogate.relu_ambiguous(**oracle_args(c1), kappa=kappa)[0]
        units = np.nonzero(amb)[0][:6]
        ok_any = False
        for bits in itertools.product([False, True], repeat=len(units)):
            mask = inter["z"] > 0
            mask[0, units] = bits
            ref = ogate.backward(**oracle_args(c1), grad_f=g1, relu_mask=mask)
            if all(grad_tol_ok(g, ref[nm])[0] for nm, g in zip(("W1", "b1", "w2", "b2", "emb"), grads)):
                ok_any = True
                break
        assert ok_any, p


def gpu_args(c):
    return (dev(c["emb"]), dev(c["lens"]), dev(c["vgene"]), dev(c["self_scores"]), dev(c["pairs"]),
            dev(c["align"]), dev(c["W1"]), dev(c["b1"]), dev(c["w2"]), dev(c["b2"]))


def oracle_args(c):
    return dict((k, c[k]) for k in ("emb", "lens", "vgene", "self_scores", "pairs", "align", "W1", "b1",
                                    "w2", "b2"))


@pytest.mark.parametrize("d,H", [(64, 64), (128, 64), (4, 16), (100, 32), (256, 128), (1024, 256), (128, 16)])
def test_forward(d, H):
    rep = synth.tiny(n_families=60, fam_size=8, seed=d + H)
    c = make_case(rep, d, H, 3000, seed=d, scale_norms=True)
    say(f"gate fwd d={d} H={H}")
    f, g = sq.gate_fwd(*gpu_args(c), return_gate=True)
    torch.cuda.synchronize()
    ref, inter = ogate.forward(**oracle_args(c), return_all=True)
    ok, err = fused_tol_ok(f.cpu().numpy(), ref)
    assert ok, err
    assert np.allclose(g.cpu().numpy(), inter["g"], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("d,H", [(64, 64), (128, 64), (100, 32), (256, 128), (4, 16)])
def test_backward(d, H):
    rep = synth.tiny(n_families=60, fam_size=8, seed=d * 3 + H)
    full = make_case(rep, d, H, 3000, seed=d + 1, scale_norms=True)
    gf_full = synth.upstream_grad(full["pairs"].shape[0], seed=d)
    c, amb = split_ambiguous(full)
    gf = np.delete(gf_full, amb)
    say(f"gate bwd d={d} H={H} (ambiguous ReLU pairs: {len(amb)})")
    grads = sq.gate_bwd(*gpu_args(c), dev(gf))
    torch.cuda.synchronize()
    ref = ogate.backward(**oracle_args(c), grad_f=gf)
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)
    check_ambiguous_pairs(full, amb, gf_full)


def test_backward_accumulates_and_skips_emb():
    rep = synth.tiny(seed=5)
    c = make_case(rep, 64, 64, 1000, seed=2)
    gf = synth.upstream_grad(c["pairs"].shape[0], seed=1)
    say("gate bwd accumulate")
    g1 = sq.gate_bwd(*gpu_args(c), dev(gf))
    g2 = sq.gate_bwd(*gpu_args(c), dev(gf), grads=tuple(x.clone() for x in g1))
    g3 = sq.gate_bwd(*gpu_args(c), dev(gf), need_emb=False)
    torch.cuda.synchronize()
    for a, b in zip(g1, g2):
        assert torch.allclose(2 * a, b, rtol=1e-6, atol=1e-7)
    for a, b in zip(g1[:4], g3[:4]):
        assert torch.allclose(a, b, rtol=1e-6, atol=1e-7)
    assert g3[4] is None


def test_gatefn_autograd_and_loss():
    rep = synth.tiny(seed=6)
    c = make_case(rep, 64, 64, 2000, seed=3)
    y = (c["family"][c["pairs"][:, 0]] == c["family"][c["pairs"][:, 1]]).astype(np.float64)
    say("GateFn autograd")
    emb = dev(c["emb"]).requires_grad_(True)
    W = [dev(c[k]).requires_grad_(True) for k in ("W1", "b1", "w2", "b2")]
    f = sq.GateFn.apply(emb, *W, dev(c["pairs"]), dev(c["align"]), dev(c["self_scores"]), dev(c["lens"]),
                        dev(c["vgene"]))
    yt = torch.as_tensor(y, dtype=torch.float32, device="cuda")
    hinge = torch.clamp(f - ogate.MARGIN, min=0)
    loss = (yt * (1 - f) ** 2 + (1 - yt) * hinge ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    f64 = ogate.forward(**oracle_args(c))
    _, gl = ogate.contrastive_loss(f64, y)
    ref = ogate.backward(**oracle_args(c), grad_f=gl)
    for name, t in zip(("emb", "W1", "b1", "w2", "b2"), (emb, *W)):
        ok, rel = grad_tol_ok(t.grad.cpu().numpy(), ref[name], rel=2e-5)
        assert ok, (name, rel)


def test_zero_norm_embedding():
    rep = synth.tiny(seed=8)
    c = make_case(rep, 64, 64, 500, seed=4)
    c["emb"] = c["emb"].copy()
    zero_rows = np.unique(c["pairs"][:20, 1])
    c["emb"][zero_rows] = 0.0
    gf = synth.upstream_grad(c["pairs"].shape[0], seed=4)
    say("gate zero-norm embeddings")
    f = sq.gate_fwd(*gpu_args(c))
    grads = sq.gate_bwd(*gpu_args(c), dev(gf))
    torch.cuda.synchronize()
    ref = ogate.forward(**oracle_args(c))
    ok, err = fused_tol_ok(f.cpu().numpy(), ref)
    assert ok, err
    rb = ogate.backward(**oracle_args(c), grad_f=gf)
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        assert np.isfinite(g.cpu().numpy()).all()
        ok, rel = grad_tol_ok(g.cpu().numpy(), rb[name])
        assert ok, (name, rel)


def test_pair_symmetry_and_empty():
    rep = synth.tiny(seed=9)
    c = make_case(rep, 64, 64, 500, seed=5)
    say("gate symmetry / empty")
    f1 = sq.gate_fwd(*gpu_args(c)).cpu().numpy()
    c2 = dict(c, pairs=np.ascontiguousarray(c["pairs"][:, ::-1]))
    f2 = sq.gate_fwd(*gpu_args(c2)).cpu().numpy()
    assert np.allclose(f1, f2, rtol=1e-6, atol=1e-7)
    c3 = dict(c, pairs=np.zeros((0, 2), np.int32), align=np.zeros(0, np.int32))
    assert sq.gate_fwd(*gpu_args(c3)).shape == (0,)


def test_gate_2p20_pairs_full_size():
    """Training workload: 2^20 family-heavy pairs of the 100k Zipf repertoire, d=128, H=64,
    forward and backward against the float64 oracle over every pair.  The few pairs with a
    ReLU pre-activation within float32 rounding of zero are checked on their own against
    either decision."""
    rep = workload("zipf100k")
    full = make_case(rep, 128, 64, 1 << 20, seed=1004, same_frac=0.7)
    gf_full = synth.upstream_grad(full["pairs"].shape[0], seed=1004)
    say(f"gate 2^20 pairs P={full['pairs'].shape[0]}")
    f = sq.gate_fwd(*gpu_args(full))
    torch.cuda.synchronize()
    ok, err = fused_tol_ok(f.cpu().numpy(), ogate.forward(**oracle_args(full)))
    assert ok, err
    c, amb = split_ambiguous(full)
    gf = np.delete(gf_full, amb)
    say(f"gate 2^20 backward, {len(amb)} ambiguous pairs set aside")
    grads = sq.gate_bwd(*gpu_args(c), dev(gf))
    torch.cuda.synchronize()
    ref = ogate.backward(**oracle_args(c), grad_f=gf)
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)
    check_ambiguous_pairs(full, amb, gf_full)


def test_backward_hub_rows():
    """Rows shared by thousands of pairs (on either side) span many workers' chunks, so both
    passes mix owned rows (plain update) with rows split between chunks (atomics)."""
    rep = synth.tiny(n_families=60, fam_size=8, seed=21)
    c = make_case(rep, 64, 64, 6000, seed=21)
    pairs = c["pairs"].copy()
    pairs[:2500, 0] = 3                       # hub as first index
    pairs[2500:4500, 1] = 7                   # hub as second index
    pairs[4500:4600] = [11, 11]               # self pairs
    c = dict(c, pairs=pairs, align=sw_oracle(rep.seqs, rep.lens, pairs, synth.load_blosum62()))
    full = c
    c, amb = split_ambiguous(full)
    gf = synth.upstream_grad(c["pairs"].shape[0], seed=21)
    say(f"gate bwd hub rows (ambiguous ReLU pairs set aside: {len(amb)})")
    grads = sq.gate_bwd(*gpu_args(c), dev(gf))
    torch.cuda.synchronize()
    ref = ogate.backward(**oracle_args(c), grad_f=gf)
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)


def test_contrastive_grad():
    """The gate's training signal against the oracle's loss and gradient (float32 kernel, the
    loss summed in float64), including out-of-range pairs (gradient 0) and P = 0."""
    rep = synth.tiny(seed=12)
    rng = np.random.default_rng(12)
    pairs = synth.random_pairs(rep.n, 5000, 12, family=rep.family, same_frac=0.5)
    f = rng.uniform(-1.0, 1.5, pairs.shape[0]).astype(np.float32)
    say("contrastive loss gradient")
    g, loss = sq.api.contrastive_grad(dev(f), dev(pairs), dev(rep.family.astype(np.int32)), 0.5)
    torch.cuda.synchronize()
    y = (rep.family[pairs[:, 0]] == rep.family[pairs[:, 1]]).astype(np.float64)
    ref_l, ref_g = ogate.contrastive_loss(f.astype(np.float64), y, 0.5)
    assert abs(loss.item() - ref_l) <= 1e-6 * abs(ref_l)
    assert np.allclose(g.cpu().numpy(), ref_g, rtol=1e-5, atol=1e-6 * np.abs(ref_g).max())
    bad = pairs.copy()
    bad[:10, 1] = rep.n + 3
    g2, _ = sq.api.contrastive_grad(dev(f), dev(bad), dev(rep.family.astype(np.int32)), 0.5)
    assert not g2.cpu().numpy()[:10].any()
    g0, l0 = sq.api.contrastive_grad(dev(f[:0]), dev(pairs[:0]), dev(rep.family.astype(np.int32)), 0.5)
    torch.cuda.synchronize()
    assert g0.shape == (0,) and l0.item() == 0.0


def _train_oracle(c, labels, margin=0.5):
    f64 = ogate.forward(**oracle_args(c))
    y = (labels[c["pairs"][:, 0]] == labels[c["pairs"][:, 1]]).astype(np.float64)
    L, gl = ogate.contrastive_loss(f64, y, margin)
    return f64, L, ogate.backward(**oracle_args(c), grad_f=gl)


@pytest.mark.parametrize("d,H", [(64, 64), (128, 64), (100, 32)])
def test_gate_train_against_oracle(d, H):
    """The fused training pass: forward values, mean contrastive loss and gradients against
    the oracle's forward, loss and backward (pairs whose ReLU decision is ambiguous at float32
    precision set aside, as for the backward)."""
    rep = synth.tiny(n_families=60, fam_size=8, seed=d + 7 * H)
    full = make_case(rep, d, H, 3000, seed=d + 2, scale_norms=True)
    c, amb = split_ambiguous(full)
    say(f"gate train d={d} H={H} (ambiguous ReLU pairs set aside: {len(amb)})")
    fused, loss, grads = sq.api.gate_train(*gpu_args(c), dev(rep.family.astype(np.int32)), 0.5)
    torch.cuda.synchronize()
    f64, L, ref = _train_oracle(c, rep.family)
    ok, err = fused_tol_ok(fused.cpu().numpy(), f64)
    assert ok, err
    assert abs(loss.item() - L) <= 1e-5 * abs(L) + 1e-7
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
        assert ok, (name, rel)


def test_gate_train_matches_separate_calls():
    """Fused pass = forward, then the contrastive gradient, then the backward: the same fused
    values bit for bit, the same loss and gradients up to summation order."""
    rep = synth.tiny(seed=31)
    c = make_case(rep, 128, 64, 4000, seed=31)
    lab = dev(rep.family.astype(np.int32))
    say("gate train vs separate calls")
    fused, loss, grads = sq.api.gate_train(*gpu_args(c), lab, 0.5)
    f2 = sq.gate_fwd(*gpu_args(c))
    gf, l2 = sq.api.contrastive_grad(f2, dev(c["pairs"]), lab, 0.5)
    g2 = sq.gate_bwd(*gpu_args(c), gf)
    torch.cuda.synchronize()
    assert torch.equal(fused, f2)
    assert abs(loss.item() - l2.item()) <= 1e-12 * abs(l2.item())
    for a, b in zip(grads, g2):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(b.abs().max()))


def test_gate_train_empty():
    rep = synth.tiny(seed=32)
    c = make_case(rep, 64, 64, 100, seed=32)
    c = dict(c, pairs=np.zeros((0, 2), np.int32), align=np.zeros(0, np.int32))
    say("gate train P=0")
    fused, loss, grads = sq.api.gate_train(*gpu_args(c), dev(rep.family.astype(np.int32)), 0.5)
    torch.cuda.synchronize()
    assert fused.shape == (0,) and loss.item() == 0.0 and not grads[4].any()
    # the writing variant with no pairs: every gradient row is written as zero
    g2 = tuple(torch.zeros_like(g) for g in grads[:4]) + (torch.full_like(grads[4], float("nan")),)
    say("gate train P=0, demb written")
    _, loss2, g2 = sq.api.gate_train(*gpu_args(c), dev(rep.family.astype(np.int32)), 0.5, grads=g2, set_demb=True)
    torch.cuda.synchronize()
    assert loss2.item() == 0.0 and not g2[4].isnan().any() and not g2[4].any()


def test_backward_sorted_and_shuffled_pairs_agree():
    """Pairs already in order of i take the backward's natural-order path (no i sort); the
    same pairs shuffled take the sorted path: gradients agree to summation order, and both
    match the oracle."""
    rep = synth.tiny(n_families=60, fam_size=8, seed=41)
    c = make_case(rep, 128, 64, 5000, seed=41)
    order = np.lexsort((c["pairs"][:, 1], c["pairs"][:, 0]))
    cs = dict(c, pairs=np.ascontiguousarray(c["pairs"][order]), align=np.ascontiguousarray(c["align"][order]))
    cs, amb = split_ambiguous(cs)
    gf = synth.upstream_grad(cs["pairs"].shape[0], seed=41)
    perm = np.random.default_rng(41).permutation(cs["pairs"].shape[0])
    cu = dict(cs, pairs=np.ascontiguousarray(cs["pairs"][perm]), align=np.ascontiguousarray(cs["align"][perm]))
    say(f"gate bwd sorted vs shuffled pairs (P={cs['pairs'].shape[0]})")
    g_sorted = sq.gate_bwd(*gpu_args(cs), dev(gf))
    g_shuf = sq.gate_bwd(*gpu_args(cu), dev(gf[perm]))
    torch.cuda.synchronize()
    ref = ogate.backward(**oracle_args(cs), grad_f=gf)
    for name, a, b in zip(("W1", "b1", "w2", "b2", "emb"), g_sorted, g_shuf):
        for g in (a, b):
            ok, rel = grad_tol_ok(g.cpu().numpy(), ref[name])
            assert ok, (name, rel)
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(b.abs().max()))


def test_gate_train_out_of_range_pairs():
    """Pairs with an index outside [0, n) are skipped: their fused value is NaN and they add
    nothing to the gradients, which equal those of the valid pairs alone (the mean loss
    still divides by every pair, so those gradients are scaled by P_valid / P)."""
    rep = synth.tiny(n_families=40, fam_size=8, seed=51)
    c = make_case(rep, 128, 64, 1500, seed=51)
    n = rep.n
    bad = np.array([[n, 0], [0, n + 5], [-1, 3], [7, -2]], np.int32)
    P = c["pairs"].shape[0]
    mixed = dict(c, pairs=np.concatenate([c["pairs"], bad]), align=np.concatenate([c["align"], np.zeros(4, np.int32)]))
    lab = dev(rep.family.astype(np.int32))
    say("gate train with out-of-range pairs")
    fused, loss, grads = sq.api.gate_train(*gpu_args(mixed), lab, 0.5)
    f_ok, l_ok, g_ok = sq.api.gate_train(*gpu_args(c), lab, 0.5)
    torch.cuda.synchronize()
    f = fused.cpu().numpy()
    assert np.isnan(f[P:]).all() and np.array_equal(f[:P], f_ok.cpu().numpy())
    scale = P / (P + 4)
    assert loss.item() == pytest.approx(l_ok.item() * scale, rel=1e-6)
    for a, b in zip(grads, g_ok):
        assert torch.allclose(a, b * scale, rtol=1e-5, atol=1e-7 * float(b.abs().max()))


def test_gate_train_no_rows():
    """n = 0 with pairs, through the C ABI with real (unused) row pointers: every pair is out
    of range, the fused values are NaN and no gradient is formed (no row is read)."""
    from paper_2602_17330_amd import _lib, api
    rep = synth.tiny(seed=52)
    c = make_case(rep, 64, 64, 50, seed=52)
    emb, lens, vgene, self_s, pairs, align_s, W1, b1, w2, b2 = gpu_args(c)
    lab = dev(rep.family.astype(np.int32))
    P, H = pairs.shape[0], W1.shape[0]
    fused = torch.zeros(P, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    grads = [torch.zeros_like(t) for t in (W1, b1, w2, b2)]
    ws = torch.empty(api.gate_bwd_workspace_bytes(H, P, 0), dtype=torch.uint8, device="cuda")
    say("gate train n=0, P=50 (C ABI)")
    api.check(_lib.lib().subquad_gate_train(
        emb.data_ptr(), 0, 64, lens.data_ptr(), vgene.data_ptr(), self_s.data_ptr(), pairs.data_ptr(),
        align_s.data_ptr(), P, W1.data_ptr(), b1.data_ptr(), w2.data_ptr(), b2.data_ptr(), H, lab.data_ptr(), 0.5,
        fused.data_ptr(), loss.data_ptr(), *[g.data_ptr() for g in grads], None, ws.data_ptr(), ws.numel(),
        torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert np.isnan(fused.cpu().numpy()).all() and loss.item() == 0.0
    assert all(not g.any() for g in grads)


@pytest.mark.parametrize("P,sorted_pairs", [(3000, False), (3000, True), (40000, True), (40000, False)])
def test_gate_train_set_writes_demb(P, sorted_pairs):
    """The writing training pass: demb starts as NaN and ends equal to the accumulating pass
    on a zeroed buffer (rows without pairs zero, rows split between chunks complete), with
    out-of-range pairs mixed in: one with i out of range, one with j out of range on a row
    that has pairs, and one on a row that has none.  Sorted pairs are walked in their own
    order (the out-of-range ones after the rest), shuffled ones through the sort."""
    rep = synth.tiny(n_families=80, fam_size=10, seed=60 + P)
    c = make_case(rep, 128, 64, P, seed=60)
    order = np.lexsort((c["pairs"][:, 1], c["pairs"][:, 0]))
    if not sorted_pairs:
        order = np.random.default_rng(P).permutation(len(order))
    c = dict(c, pairs=np.ascontiguousarray(c["pairs"][order]), align=np.ascontiguousarray(c["align"][order]))
    n = rep.n
    lone = int(np.setdiff1d(np.arange(n), c["pairs"][:, 0])[0])  # a row with no pair as i
    bad = np.array([[n, 0], [2, n + 1], [lone, -1]], np.int32)
    c = dict(c, pairs=np.concatenate([c["pairs"], bad]), align=np.concatenate([c["align"], np.zeros(3, np.int32)]))
    lab = dev(rep.family.astype(np.int32))
    args = gpu_args(c)
    say(f"gate train, demb written (P={P}, sorted={sorted_pairs})")
    f1, l1, g1 = sq.api.gate_train(*args, lab, 0.5)
    g2 = tuple(torch.zeros_like(g) for g in g1[:4]) + (torch.full_like(g1[4], float("nan")),)
    f2, l2, g2 = sq.api.gate_train(*args, lab, 0.5, grads=g2, set_demb=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(f1, nan=-7.0), torch.nan_to_num(f2, nan=-7.0))
    assert l1.item() == l2.item()
    assert not torch.isnan(g2[4]).any()
    touched = np.zeros(n, bool)
    ok = (c["pairs"] >= 0).all(axis=1) & (c["pairs"] < n).all(axis=1)
    touched[c["pairs"][ok].ravel()] = True
    assert not g2[4][torch.from_numpy(~touched).cuda()].any()
    for a, b in zip(g1, g2):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(a.abs().max()))


def _rep1m_train_case(P, seed):
    """P candidate pairs of the 1M-sequence workload (a seeded sample of the oracle's
    candidate set, in its sorted order), their oracle alignment scores, d = 128, H = 64."""
    rep = workload("rep1m")
    cand = oracle_candidates("rep1m")
    pick = np.sort(synth.sample_rows(cand.shape[0], P, seed))
    S = synth.load_blosum62()
    W1, b1, w2, b2 = synth.gate_params(64)
    return rep, dict(emb=synth.embeddings(rep.seqs, rep.lens, 128), lens=rep.lens, vgene=rep.vgene,
                     self_scores=osw.self_scores(rep.seqs, rep.lens, S),
                     pairs=np.ascontiguousarray(cand[pick].astype(np.int32)),
                     align=np.ascontiguousarray(oracle_scores("rep1m")[pick]), W1=W1, b1=b1, w2=w2, b2=b2)


@pytest.mark.parametrize("P,groups_per_cu", [(1 << 20, None), (1_500_000, 1)])
def test_gate_train_set_rep1m_2p20_against_oracle(P, groups_per_cu):
    """The writing training pass the benchmark step runs, on 2^20 of the 1M workload's
    candidate pairs (each 16-lane group walks tens of prefetched batches): fused values of
    every pair, the mean loss, the weight gradients and every row of the embedding gradient
    against the float64 oracle.  Hidden units within float32 rounding of the ReLU kink widen
    the bounds by exactly what flipping each of them changes.  With one lane group per CU
    (256 groups) 1.5M pairs exceed 256 chunks of the 4096-pair cap: every group walks two
    chunks in rounds and the second backward pass takes its looping form."""
    from paper_2602_17330_amd import autotune
    rep, c = _rep1m_train_case(P, 1005)
    lab = rep.family.astype(np.int32)
    args = gpu_args(c)
    W = args[6:]
    g0 = tuple(torch.zeros_like(w) for w in W) + (torch.full_like(args[0], float("nan")),)
    say(f"gate train set rep1m P={c['pairs'].shape[0]} groups_per_cu={groups_per_cu}")
    old_knob = autotune.get_knob("gate_groups_per_cu")
    try:
        if groups_per_cu:
            autotune.set_knob("gate_groups_per_cu", groups_per_cu)
        fused, loss, grads = sq.api.gate_train(*args, dev(lab), 0.5, grads=g0, set_demb=True)
        torch.cuda.synchronize()
    finally:
        autotune.set_knob("gate_groups_per_cu", old_knob)
    fused = fused.cpu().numpy()
    grads = [g.cpu().numpy() for g in grads]
    say("gate train set rep1m: oracle forward")
    oa = oracle_args(c)
    f64 = ogate.forward(**oa)
    ok, err = fused_tol_ok(fused, f64)
    assert ok, err
    y = (lab[c["pairs"][:, 0]] == lab[c["pairs"][:, 1]]).astype(np.float64)
    L, gl = ogate.contrastive_loss(f64, y, 0.5)
    assert abs(loss.item() - L) <= 1e-5 * abs(L) + 1e-7
    say("gate train set rep1m: oracle backward")
    ref = gate_backward_chunked(oa, gl)
    n_amb, ew, nw = ambiguous_flip_bounds(oa, gl)
    say(f"gate train set rep1m: {n_amb} ambiguous ReLU decisions")
    assert not np.isnan(grads[4]).any()
    for name, g in zip(("W1", "b1", "w2", "b2", "emb"), grads):
        ok, rel = grads_ok_widened(g, ref[name], ew[name], nw[name])
        assert ok, (name, rel)


@pytest.mark.parametrize("sorted_pairs", [True, False])
def test_gate_train_set_rep1m_2p20_writes_demb(sorted_pairs):
    """At 2^20 candidate pairs of the 1M workload, sorted and shuffled, with out-of-range
    pairs mixed in: the writing pass on a NaN-filled gradient equals the accumulating pass on
    zeros (rows without pairs zero, rows split between chunks complete)."""
    rep, c = _rep1m_train_case(1 << 20, 1006)
    n = rep.n
    order = np.arange(c["pairs"].shape[0]) if sorted_pairs else np.random.default_rng(7).permutation(
        c["pairs"].shape[0])
    lone = int(np.setdiff1d(np.arange(n), c["pairs"][:, 0])[0])   # a row with no pair as i
    bad = np.array([[n, 0], [2, n + 1], [lone, -1]], np.int32)
    c = dict(c, pairs=np.ascontiguousarray(np.concatenate([c["pairs"][order], bad])),
             align=np.ascontiguousarray(np.concatenate([c["align"][order], np.zeros(3, np.int32)])))
    lab = dev(rep.family.astype(np.int32))
    args = gpu_args(c)
    say(f"gate train set vs accumulate rep1m P={c['pairs'].shape[0]} sorted={sorted_pairs}")
    f1, l1, g1 = sq.api.gate_train(*args, lab, 0.5)
    g2 = tuple(torch.zeros_like(g) for g in g1[:4]) + (torch.full_like(g1[4], float("nan")),)
    f2, l2, g2 = sq.api.gate_train(*args, lab, 0.5, grads=g2, set_demb=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(f1, nan=-7.0), torch.nan_to_num(f2, nan=-7.0))
    assert np.isnan(f2[-3:].cpu().numpy()).all()
    assert l1.item() == l2.item()
    assert not torch.isnan(g2[4]).any()
    touched = np.zeros(n, bool)
    ok = (c["pairs"] >= 0).all(axis=1) & (c["pairs"] < n).all(axis=1)
    touched[c["pairs"][ok].ravel()] = True
    assert not g2[4][torch.from_numpy(~touched).cuda()].any()
    for a, b in zip(g1, g2):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(a.abs().max()))


def test_gate_train_set_8m_shuffled_pairs_sorted_by_i():
    """8M pairs of the 1M-sequence workload (about 2,000 sort tiles: more than the chip holds
    blocks of the i sort at once, so that sort loops over its tiles), shuffled, against the
    same pairs in order of i (whose i sort is empty): fused values equal pair by pair, the
    loss and every gradient equal to summation order."""
    rep = workload("rep1m")
    n = rep.n
    pairs = synth.random_pairs(n, 9_700_000, 31, family=rep.family, same_frac=0.5)  # (duplicates dropped)
    P = pairs.shape[0]
    assert P >= 8_000_000
    rng = np.random.default_rng(31)
    align = rng.integers(0, 120, P).astype(np.int32)
    W1, b1, w2, b2 = synth.gate_params(64)
    S = synth.load_blosum62()
    c = dict(emb=synth.embeddings(rep.seqs, rep.lens, 128), lens=rep.lens, vgene=rep.vgene,
             self_scores=osw.self_scores(rep.seqs, rep.lens, S), pairs=pairs, align=align,
             W1=W1, b1=b1, w2=w2, b2=b2)
    perm = rng.permutation(P)
    cu = dict(c, pairs=np.ascontiguousarray(pairs[perm]), align=np.ascontiguousarray(align[perm]))
    lab = dev(rep.family.astype(np.int32))
    say(f"gate train set P={P}: pairs in order of i, then shuffled")
    runs = []
    for case in (c, cu):
        args = gpu_args(case)
        g0 = tuple(torch.zeros_like(w) for w in args[6:]) + (torch.full_like(args[0], float("nan")),)
        f, loss, g = sq.api.gate_train(*args, lab, 0.5, grads=g0, set_demb=True)
        torch.cuda.synchronize()
        runs.append((f[:P].cpu().numpy(), loss.item(), [x.cpu() for x in g]))
    (f_s, l_s, g_s), (f_u, l_u, g_u) = runs
    assert np.array_equal(f_s[perm], f_u)
    assert abs(l_s - l_u) <= 1e-12 * abs(l_s)
    assert not torch.isnan(g_u[4]).any()
    for a, b in zip(g_s, g_u):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(a.abs().max()))
