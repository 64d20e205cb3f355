"""Pins for the gate oracle: closed forms of the fusion, the two-channel softmax identity,
central finite differences (the scheme of the paper's Appendix B risk-gradient estimate)
and torch float64 autograd of an independently written forward."""
import numpy as np
import pytest
import torch

import synth
from oracle import gate
from oracle import sw


@pytest.fixture(scope="module")
def case(blosum62):
    r = synth.tiny(n_families=30, fam_size=6, seed=13)
    emb = synth.embeddings(r.seqs, r.lens, 32).astype(np.float64)
    rng = np.random.default_rng(0)
    emb = emb * rng.uniform(0.5, 2.0, (r.n, 1))            # non-unit norms exercise the cosine
    pairs = synth.random_pairs(r.n, 400, 1, family=r.family)
    align = sw.scores_pairs(r.seqs, r.lens, pairs, blosum62)
    self_s = sw.self_scores(r.seqs, r.lens, blosum62)
    W1, b1, w2, b2 = [x.astype(np.float64) for x in synth.gate_params(16, seed=3)]
    return dict(emb=emb, lens=r.lens, vgene=r.vgene, self_scores=self_s, pairs=pairs, align=align,
                W1=W1, b1=b1, w2=w2 * 8, b2=b2, family=r.family)


def _fwd(c, **over):
    a = dict(c)
    a.update(over)
    a.pop("family")
    return gate.forward(**a)


def test_zero_weights_average(case):
    H = case["W1"].shape[0]
    f = _fwd(case, W1=np.zeros((H, 4)), b1=np.zeros(H), w2=np.zeros(H), b2=np.zeros(1))
    ft = gate.features(case["emb"], case["lens"], case["vgene"], case["self_scores"],
                       case["pairs"], case["align"])
    assert np.allclose(f, 0.5 * (ft["s"] + ft["c"]), rtol=0, atol=1e-15)


def test_saturated_gate_selects_a_channel(case):
    H = case["W1"].shape[0]
    ft = gate.features(case["emb"], case["lens"], case["vgene"], case["self_scores"],
                       case["pairs"], case["align"])
    f_hi = _fwd(case, w2=np.zeros(H), b2=np.array([50.0]))
    f_lo = _fwd(case, w2=np.zeros(H), b2=np.array([-50.0]))
    assert np.allclose(f_hi, ft["s"], rtol=0, atol=1e-20 + 1e-15)
    assert np.allclose(f_lo, ft["c"], rtol=0, atol=1e-20 + 1e-15)


def test_features_ranges(case):
    ft = gate.features(case["emb"], case["lens"], case["vgene"], case["self_scores"],
                       case["pairs"], case["align"])
    assert (ft["s"] >= 0).all() and (ft["s"] <= 1 + 1e-15).all()
    assert (np.abs(ft["c"]) <= 1 + 1e-12).all()
    same = np.stack([np.arange(10), np.arange(10)], 1)
    f2 = gate.features(case["emb"], case["lens"], case["vgene"], case["self_scores"], same,
                       case["self_scores"][:10])
    assert np.allclose(f2["s"], 1.0) and np.allclose(f2["c"], 1.0)


def test_softmax_matches_sigmoid(case):
    f, a = _fwd(case, return_all=True)
    g = 1.0 / (1.0 + np.exp(-a["u"]))
    assert np.allclose(a["g"], g, rtol=1e-14, atol=1e-15)
    assert np.allclose(f, g * a["s"] + (1 - g) * a["c"], rtol=1e-13, atol=1e-15)


def test_pair_symmetry(case):
    swp = case["pairs"][:, ::-1].copy()
    assert np.allclose(_fwd(case), _fwd(case, pairs=swp), rtol=1e-14, atol=1e-15)


def _torch_forward(emb, lens, vgene, self_s, pairs, align, W1, b1, w2, b2):
    """Independent torch float64 transcription of the fused score."""
    i = torch.as_tensor(pairs[:, 0], dtype=torch.long)
    j = torch.as_tensor(pairs[:, 1], dtype=torch.long)
    S = torch.as_tensor(self_s, dtype=torch.float64)
    s = torch.as_tensor(align, dtype=torch.float64) / torch.sqrt(S[i] * S[j])
    c = torch.nn.functional.cosine_similarity(emb[i], emb[j], dim=1, eps=0.0)
    L = torch.as_tensor(lens, dtype=torch.float64)
    V = torch.as_tensor(vgene)
    x = torch.stack([s, c, (L[i] - L[j]).abs(), (V[i] == V[j]).double()], 1)
    h = torch.relu(x @ W1.T + b1)
    u = h @ w2 + b2
    w = torch.softmax(torch.stack([u, torch.zeros_like(u)], 1), 1)
    return w[:, 0] * s + w[:, 1] * c


def test_backward_against_torch_autograd(case):
    rng = np.random.default_rng(7)
    gf = rng.standard_normal(case["pairs"].shape[0])
    ref = {k: torch.tensor(case[k], dtype=torch.float64, requires_grad=True)
           for k in ("emb", "W1", "b1", "w2", "b2")}
    f = _torch_forward(ref["emb"], case["lens"], case["vgene"], case["self_scores"], case["pairs"],
                       case["align"], ref["W1"], ref["b1"], ref["w2"], ref["b2"])
    (f * torch.as_tensor(gf)).sum().backward()
    a = dict(case)
    a.pop("family")
    got = gate.backward(**a, grad_f=gf)
    assert np.allclose(got["f"], f.detach().numpy(), rtol=1e-13, atol=1e-15)
    for k in ("emb", "W1", "b1", "w2", "b2"):
        assert np.allclose(got[k], ref[k].grad.numpy(), rtol=1e-11, atol=1e-13), k


def test_backward_finite_differences(case):
    """Central differences (L(t + h) - L(t - h)) / 2h of L = sum gf * f, h = 1e-6."""
    rng = np.random.default_rng(8)
    gf = rng.standard_normal(case["pairs"].shape[0])
    a = dict(case)
    a.pop("family")
    got = gate.backward(**a, grad_f=gf)
    _, inter = gate.forward(**a, return_all=True)
    if np.abs(inter["z"]).min() < 1e-4:
        pytest.skip("a pre-activation sits on the ReLU kink")
    h = 1e-6

    def L(**over):
        return float((gf * _fwd(case, **over)).sum())

    for name in ("W1", "b1", "w2", "b2"):
        base = case[name]
        for idx in list(np.ndindex(base.shape))[:12]:
            p, m = base.copy(), base.copy()
            p[idx] += h
            m[idx] -= h
            fd = (L(**{name: p}) - L(**{name: m})) / (2 * h)
            assert abs(fd - got[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
    E = case["emb"]
    for (r_, k_) in [(0, 0), (5, 3), (17, 31), (int(case["pairs"][0, 1]), 7)]:
        p, m = E.copy(), E.copy()
        p[r_, k_] += h
        m[r_, k_] -= h
        fd = (L(emb=p) - L(emb=m)) / (2 * h)
        assert abs(fd - got["emb"][r_, k_]) <= 1e-6 * max(1.0, abs(fd))


def test_contrastive_loss_gradient():
    rng = np.random.default_rng(9)
    f = rng.uniform(-1, 1, 50)
    y = (rng.random(50) < 0.5).astype(float)
    _, g = gate.contrastive_loss(f, y)
    h = 1e-6
    for k in range(50):
        fp, fm = f.copy(), f.copy()
        fp[k] += h
        fm[k] -= h
        fd = (gate.contrastive_loss(fp, y)[0] - gate.contrastive_loss(fm, y)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8


def test_relu_mask_override(case):
    """An explicit ReLU decision equal to z > 0 changes nothing; flipping one (pair, unit)
    changes dW1 by exactly that unit's chain-rule term."""
    a = dict(case)
    a.pop("family")
    gf = np.random.default_rng(3).standard_normal(case["pairs"].shape[0])
    base = gate.backward(**a, grad_f=gf)
    _, inter = gate.forward(**a, return_all=True)
    mask = inter["z"] > 0
    same = gate.backward(**a, grad_f=gf, relu_mask=mask)
    for k in ("W1", "b1", "w2", "b2", "emb"):
        assert np.array_equal(base[k], same[k])
    p, k = 5, 3
    flipped = mask.copy()
    flipped[p, k] = ~flipped[p, k]
    alt = gate.backward(**a, grad_f=gf, relu_mask=flipped)
    g = inter["g"][p]
    ubar = gf[p] * (inter["s"][p] - inter["c"][p]) * g * (1 - g)
    term = ubar * case["w2"][k] * inter["X"][p]
    sign = 1.0 if flipped[p, k] else -1.0
    assert np.allclose(alt["W1"][k] - base["W1"][k], sign * term, rtol=1e-12, atol=1e-15)
    amb = gate.relu_ambiguous(**a, kappa=1.0)
    assert amb.all()                       # every unit is within 1x its own scale of zero
    assert not gate.relu_ambiguous(**a, kappa=0.0).any() or (inter["z"] == 0).any()
