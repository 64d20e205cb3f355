"""Oracle: per-pair dynamic affinity fusion (forward and backward), float64.

Paper: Sec. 3.6, Eq. (wm) and Eq. (afused) -- per pair (i, j), channel scores g^(m) from a
small two-layer MLP are normalised by a softmax into weights w^(m), and the fused affinity
is sum_m w^(m) a^(m). Sec. 3.3, Eq. (alpha) gives the sigmoid channel weighting.
Algorithm 1 (affinity computation) evaluates this for every candidate pair.

Readings where the paper is silent:
  * two channels: a^(1) = s_ij, the alignment score normalised by the geometric mean of the
    self-scores, s_ij = A_ij / sqrt(S_i S_j); a^(2) = c_ij, the cosine of the embeddings;
  * the MLP reads x = (s_ij, c_ij, |L_i - L_j|, [V_i == V_j]) (raw values), has H ReLU
    hidden units (ReLU is the hidden activation the paper uses for its meta-controller MLP,
    Appendix B, meta-controller algorithm) and outputs one logit u; the channel logits are
    (u, 0), so the softmax weights are (sigmoid(u), 1 - sigmoid(u));
  * ReLU'(0) = 0; a cosine with a zero-norm operand is 0 with zero gradient;
  * gradients flow to the MLP weights and the embeddings only (s, |dL| and the V-gene bit
    come from integers).
"""
from __future__ import annotations

import numpy as np


def features(emb, lens, vgene, self_scores, pairs, align):
    """Per-pair inputs: s, c, delta, v and the embedding norms (float64)."""
    E = np.asarray(emb, dtype=np.float64)
    i = np.asarray(pairs)[:, 0].astype(np.int64)
    j = np.asarray(pairs)[:, 1].astype(np.int64)
    S = np.asarray(self_scores, dtype=np.float64)
    s = np.asarray(align, dtype=np.float64) / np.sqrt(S[i] * S[j])
    ni = np.linalg.norm(E[i], axis=1)
    nj = np.linalg.norm(E[j], axis=1)
    dot = np.einsum("pk,pk->p", E[i], E[j])
    den = ni * nj
    ok = den >= 1e-12
    c = np.where(ok, dot / np.where(ok, den, 1.0), 0.0)
    L = np.asarray(lens, dtype=np.float64)
    delta = np.abs(L[i] - L[j])
    V = np.asarray(vgene)
    v = (V[i] == V[j]).astype(np.float64)
    return dict(i=i, j=j, s=s, c=c, delta=delta, v=v, ni=ni, nj=nj, ok=ok)


def forward(emb, lens, vgene, self_scores, pairs, align, W1, b1, w2, b2, return_all=False):
    """Fused affinity f[P] (float64); with ``return_all`` also the intermediates."""
    ft = features(emb, lens, vgene, self_scores, pairs, align)
    X = np.stack([ft["s"], ft["c"], ft["delta"], ft["v"]], axis=1)          # [P, 4]
    W1 = np.asarray(W1, np.float64)
    z = X @ W1.T + np.asarray(b1, np.float64)[None, :]                      # [P, H]
    h = np.maximum(z, 0.0)
    u = h @ np.asarray(w2, np.float64) + float(np.asarray(b2, np.float64).reshape(-1)[0])
    # softmax over the two channel logits (u, 0), Eq. (wm); fused sum, Eq. (afused)
    logits = np.stack([u, np.zeros_like(u)], axis=1)
    m = logits.max(axis=1, keepdims=True)
    w = np.exp(logits - m)
    w /= w.sum(axis=1, keepdims=True)
    f = w[:, 0] * ft["s"] + w[:, 1] * ft["c"]
    if return_all:
        return f, dict(ft, X=X, z=z, h=h, u=u, g=w[:, 0])
    return f


def relu_ambiguous(emb, lens, vgene, self_scores, pairs, align, W1, b1, w2, b2, kappa=1e-6):
    """bool[P, H]: hidden units whose pre-activation z lies within kappa * (|W1| |x| + |b1|) of
    0, i.e. where a float32 evaluation of z may take the other side of the ReLU kink."""
    _, a = forward(emb, lens, vgene, self_scores, pairs, align, W1, b1, w2, b2, return_all=True)
    scale = np.abs(a["X"]) @ np.abs(np.asarray(W1, np.float64)).T + np.abs(np.asarray(b1, np.float64))
    return np.abs(a["z"]) <= kappa * scale


def backward(emb, lens, vgene, self_scores, pairs, align, W1, b1, w2, b2, grad_f, relu_mask=None):
    """Gradients of sum_p grad_f[p] * f[p] w.r.t. W1, b1, w2, b2 and the embeddings,
    by the chain rule through the forward above (float64).  ``relu_mask`` (bool[P, H])
    replaces the decision z > 0 of ReLU'(z) when given (a decision taken elsewhere)."""
    f, a = forward(emb, lens, vgene, self_scores, pairs, align, W1, b1, w2, b2, return_all=True)
    gf = np.asarray(grad_f, dtype=np.float64)
    g = a["g"]
    s, c = a["s"], a["c"]
    # f = g s + (1 - g) c
    g_bar = gf * (s - c)
    u_bar = g_bar * g * (1.0 - g)
    dw2 = a["h"].T @ u_bar
    db2 = np.array([u_bar.sum()])
    h_bar = u_bar[:, None] * np.asarray(w2, np.float64)[None, :]
    mask = (a["z"] > 0.0) if relu_mask is None else np.asarray(relu_mask, dtype=bool)
    z_bar = h_bar * mask
    dW1 = z_bar.T @ a["X"]
    db1 = z_bar.sum(axis=0)
    x_bar = z_bar @ np.asarray(W1, np.float64)                                # [P, 4]
    c_bar = gf * (1.0 - g) + x_bar[:, 1]
    c_bar = np.where(a["ok"], c_bar, 0.0)
    E = np.asarray(emb, dtype=np.float64)
    i, j = a["i"], a["j"]
    ni, nj = a["ni"], a["nj"]
    safe_i = np.where(a["ok"], ni, 1.0)
    safe_j = np.where(a["ok"], nj, 1.0)
    dc_dei = E[j] / (safe_i * safe_j)[:, None] - (c / safe_i ** 2)[:, None] * E[i]
    dc_dej = E[i] / (safe_i * safe_j)[:, None] - (c / safe_j ** 2)[:, None] * E[j]
    dE = np.zeros_like(E)
    np.add.at(dE, i, c_bar[:, None] * dc_dei)
    np.add.at(dE, j, c_bar[:, None] * dc_dej)
    return dict(W1=dW1, b1=db1, w2=dw2, b2=db2, emb=dE, f=f)


MARGIN = 0.5


def contrastive_loss(f, y, margin: float = MARGIN):
    """Margin contrastive loss in similarity form (Hadsell, Chopra & LeCun 2006):
    mean of y (1 - f)^2 + (1 - y) max(0, f - margin)^2. Returns (loss, dL/df)."""
    f = np.asarray(f, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    P = max(1, f.shape[0])
    hinge = np.maximum(0.0, f - margin)
    loss = (y * (1.0 - f) ** 2 + (1.0 - y) * hinge ** 2).sum() / P
    grad = (-2.0 * y * (1.0 - f) + 2.0 * (1.0 - y) * hinge) / P
    return loss, grad


# ----------------------------------------------------------------------------- M channels
#
# Eq. (wm)/(afused) for M channels: one shared hidden layer, one logit per channel,
#   z = W1 x + b1 (H), h = relu(z), g = W2 h + b2 (M), w = softmax(g), f = sum_m w_m a_m,
# with channels a = (s, c, e) (alignment, embedding cosine, edit-distance similarity) and
# features x = (s, c, e, |L_i - L_j|, [V_i == V_j]).  Reading: the paper's g^(m) share the
# hidden layer of one two-layer MLP with M outputs.

def forward_m(emb, lens, vgene, self_scores, pairs, align, edit_sim, W1, b1, W2, b2, return_all=False):
    ft = features(emb, lens, vgene, self_scores, pairs, align)
    e = np.asarray(edit_sim, dtype=np.float64)
    A = np.stack([ft["s"], ft["c"], e], axis=1)                               # [P, 3]
    X = np.stack([ft["s"], ft["c"], e, ft["delta"], ft["v"]], axis=1)        # [P, 5]
    z = X @ np.asarray(W1, np.float64).T + np.asarray(b1, np.float64)[None, :]
    h = np.maximum(z, 0.0)
    g = h @ np.asarray(W2, np.float64).T + np.asarray(b2, np.float64)[None, :]  # [P, M]
    g = g - g.max(axis=1, keepdims=True)
    w = np.exp(g)
    w /= w.sum(axis=1, keepdims=True)
    f = (w * A).sum(axis=1)
    if return_all:
        return f, dict(ft, A=A, X=X, z=z, h=h, w=w)
    return f


def backward_m(emb, lens, vgene, self_scores, pairs, align, edit_sim, W1, b1, W2, b2, grad_f, relu_mask=None):
    f, a = forward_m(emb, lens, vgene, self_scores, pairs, align, edit_sim, W1, b1, W2, b2, return_all=True)
    gf = np.asarray(grad_f, dtype=np.float64)
    w, A = a["w"], a["A"]
    g_bar = gf[:, None] * w * (A - f[:, None])                                # d f / d g_m
    dW2 = g_bar.T @ a["h"]
    db2 = g_bar.sum(axis=0)
    h_bar = g_bar @ np.asarray(W2, np.float64)
    mask = (a["z"] > 0.0) if relu_mask is None else np.asarray(relu_mask, dtype=bool)
    z_bar = h_bar * mask
    dW1 = z_bar.T @ a["X"]
    db1 = z_bar.sum(axis=0)
    x_bar = z_bar @ np.asarray(W1, np.float64)                                # [P, 5]
    c_bar = gf * w[:, 1] + x_bar[:, 1]
    c_bar = np.where(a["ok"], c_bar, 0.0)
    E = np.asarray(emb, dtype=np.float64)
    i, j = a["i"], a["j"]
    safe_i = np.where(a["ok"], a["ni"], 1.0)
    safe_j = np.where(a["ok"], a["nj"], 1.0)
    c = a["c"]
    dc_dei = E[j] / (safe_i * safe_j)[:, None] - (c / safe_i ** 2)[:, None] * E[i]
    dc_dej = E[i] / (safe_i * safe_j)[:, None] - (c / safe_j ** 2)[:, None] * E[j]
    dE = np.zeros_like(E)
    np.add.at(dE, i, c_bar[:, None] * dc_dei)
    np.add.at(dE, j, c_bar[:, None] * dc_dej)
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2, emb=dE, f=f)


def relu_ambiguous_m(emb, lens, vgene, self_scores, pairs, align, edit_sim, W1, b1, W2, b2, kappa=1e-6):
    _, a = forward_m(emb, lens, vgene, self_scores, pairs, align, edit_sim, W1, b1, W2, b2, return_all=True)
    scale = np.abs(a["X"]) @ np.abs(np.asarray(W1, np.float64)).T + np.abs(np.asarray(b1, np.float64))
    return np.abs(a["z"]) <= kappa * scale
