"""Pins for the edit-distance channel and the M-channel gate oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import edit, gate, sw


@pytest.fixture(scope="module")
def C(blosum62):
    return edit.cost_matrix(blosum62)


def test_cost_matrix(C, blosum62):
    assert (np.diag(C) == 0).all() and (C == C.T).all()
    idx = synth.ALPHABET.index
    assert C[idx("I"), idx("V")] == 1 and C[idx("W"), idx("N")] == 2 and C[idx("K"), idx("S")] == 2


def test_classic_levenshtein(C):
    # KITTEN -> SITTING: K->S (BLOSUM62 0: not conservative), E->I, +G: 3 unit edits
    a, L = synth.encode(["KITTEN", "SITTING"], 16)
    assert edit.distance_py(list(a[0, :6]), list(a[1, :7]), C) == 2 * 3


def test_bruteforce_tiny(C):
    rng = np.random.default_rng(1)
    for _ in range(60):
        a = list(rng.integers(0, 20, rng.integers(1, 6)))
        b = list(rng.integers(0, 20, rng.integers(1, 6)))
        ref = edit.distance_bruteforce(a, b, C)
        assert edit.distance_py(a, b, C) == ref


def test_c_matches_python_and_metric(C):
    r = synth.tiny(seed=4)
    pairs = synth.random_pairs(r.n, 400, 2, family=r.family)
    d = edit.distances_pairs(r.seqs, r.lens, pairs, C)
    for p in range(0, pairs.shape[0], 17):
        i, j = pairs[p]
        assert d[p] == edit.distance_py(list(r.seqs[i, :r.lens[i]]), list(r.seqs[j, :r.lens[j]]), C)
    rng = np.random.default_rng(5)
    for _ in range(100):        # symmetry, identity, triangle inequality
        a, b, c = (list(rng.integers(0, 20, rng.integers(1, 12))) for _ in range(3))
        dab, dba = edit.distance_py(a, b, C), edit.distance_py(b, a, C)
        assert dab == dba and edit.distance_py(a, a, C) == 0
        assert edit.distance_py(a, c, C) <= dab + edit.distance_py(b, c, C)
        assert abs(len(a) - len(b)) * 2 <= dab <= 2 * max(len(a), len(b))
    sim = edit.similarity(d, r.lens, pairs)
    assert (sim >= 0).all() and (sim <= 1).all()


@pytest.fixture(scope="module")
def mcase(blosum62, C):
    r = synth.tiny(n_families=30, fam_size=6, seed=17)
    emb = synth.embeddings(r.seqs, r.lens, 32).astype(np.float64)
    emb = emb * np.random.default_rng(0).uniform(0.5, 2.0, (r.n, 1))
    pairs = synth.random_pairs(r.n, 300, 1, family=r.family)
    align = sw.scores_pairs(r.seqs, r.lens, pairs, blosum62)
    e = edit.similarity(edit.distances_pairs(r.seqs, r.lens, pairs, C), r.lens, pairs)
    rng = np.random.default_rng(2)
    H = 16
    return dict(emb=emb, lens=r.lens, vgene=r.vgene, self_scores=sw.self_scores(r.seqs, r.lens, blosum62),
                pairs=pairs, align=align, edit_sim=e, W1=rng.uniform(-0.5, 0.5, (H, 5)),
                b1=rng.uniform(-0.5, 0.5, H), W2=rng.uniform(-1, 1, (3, H)), b2=rng.uniform(-0.3, 0.3, 3))


def test_m_gate_reduces_to_two_channels(mcase):
    """Third logit at -inf and the edit feature unused: the M-channel gate is the
    two-channel gate with logits (g1 - g2, 0)."""
    c = dict(mcase)
    W1 = c["W1"].copy()
    W1[:, 2] = 0.0
    W2 = c["W2"].copy()
    b2 = c["b2"].copy()
    b2[2] = -1e9
    fm = gate.forward_m(**dict(c, W1=W1, W2=W2, b2=b2))
    W1_2 = W1[:, [0, 1, 3, 4]]
    f2 = gate.forward(c["emb"], c["lens"], c["vgene"], c["self_scores"], c["pairs"], c["align"], W1_2, c["b1"],
                      W2[0] - W2[1], np.array([b2[0] - b2[1]]))
    assert np.allclose(fm, f2, rtol=1e-12, atol=1e-14)


def test_m_gate_zero_weights_is_mean(mcase):
    c = dict(mcase)
    H = c["W1"].shape[0]
    f, a = gate.forward_m(**dict(c, W1=np.zeros((H, 5)), b1=np.zeros(H), W2=np.zeros((3, H)), b2=np.zeros(3)),
                          return_all=True)
    assert np.allclose(f, a["A"].mean(axis=1), rtol=0, atol=1e-15)


def test_m_gate_backward_autograd(mcase):
    c = mcase
    gf = np.random.default_rng(3).standard_normal(c["pairs"].shape[0])
    T = {k: torch.tensor(c[k], dtype=torch.float64, requires_grad=True) for k in ("emb", "W1", "b1", "W2", "b2")}
    i = torch.as_tensor(c["pairs"][:, 0], dtype=torch.long)
    j = torch.as_tensor(c["pairs"][:, 1], dtype=torch.long)
    S = torch.as_tensor(c["self_scores"], dtype=torch.float64)
    s = torch.as_tensor(c["align"], dtype=torch.float64) / torch.sqrt(S[i] * S[j])
    cs = torch.nn.functional.cosine_similarity(T["emb"][i], T["emb"][j], dim=1, eps=0.0)
    e = torch.as_tensor(c["edit_sim"])
    L = torch.as_tensor(c["lens"], dtype=torch.float64)
    V = torch.as_tensor(c["vgene"])
    x = torch.stack([s, cs, e, (L[i] - L[j]).abs(), (V[i] == V[j]).double()], 1)
    h = torch.relu(x @ T["W1"].T + T["b1"])
    w = torch.softmax(h @ T["W2"].T + T["b2"], dim=1)
    f = (w * torch.stack([s, cs, e], 1)).sum(1)
    (f * torch.as_tensor(gf)).sum().backward()
    got = gate.backward_m(**c, grad_f=gf)
    assert np.allclose(got["f"], f.detach().numpy(), rtol=1e-13, atol=1e-15)
    for k in ("emb", "W1", "b1", "W2", "b2"):
        assert np.allclose(got[k], T[k].grad.numpy(), rtol=1e-11, atol=1e-13), k


def test_bruteforce_asymmetric_costs():
    """An asymmetric cost matrix: cost[a][b] for a residue of the first string against one of
    the second; the C loop (both orders of a pair) equals the enumeration."""
    rng = np.random.default_rng(4)
    Ca = rng.integers(0, 5, (20, 20)).astype(np.int8)
    np.fill_diagonal(Ca, 0)
    differ = 0
    for _ in range(40):
        a = [int(x) % 5 for x in rng.integers(0, 20, rng.integers(1, 6))]
        b = [int(x) % 5 for x in rng.integers(0, 20, rng.integers(1, 6))]
        ref_ab, ref_ba = edit.distance_bruteforce(a, b, Ca, 3), edit.distance_bruteforce(b, a, Ca, 3)
        seqs = np.full((2, 8), 0xFF, np.uint8)
        seqs[0, : len(a)], seqs[1, : len(b)] = a, b
        lens = np.array([len(a), len(b)], np.int32)
        got = edit.distances_pairs(seqs, lens, np.array([[0, 1], [1, 0]], np.int32), Ca, 3)
        assert list(got) == [ref_ab, ref_ba] and edit.distance_py(a, b, Ca, 3) == ref_ab
        differ += ref_ab != ref_ba
    assert differ > 0
