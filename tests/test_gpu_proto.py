"""GPU prototype-contrastive loss (Eq. (pc), Eq. (proto)) against the float64 oracle.

Tolerances, derived from the float32 arithmetic (u = 2^-24) against the float64 oracle:
  * prototypes: |dP| <= 1e-6 max|P| (a float64 class sum rounded once);
  * logits <e, p> / tau are float32 dot products over d terms, off by about sqrt(d) u |e||p| / tau;
    a row loss log(1 + sum_{c != y} exp(z_c - z_y)) inherits at most twice that, so per row
    |d| <= 1e-5 |ref| + 4 sqrt(d) u max|e| max|p| / tau, and the total loss the sum of those;
  * gradients: normwise <= 1e-5 ||ref||, and per element <= 1e-5 |ref| + f max|ref| with
    f = max(1e-6, 2 sqrt(K) u), K = max(B, C): every gradient element is a float32 sum of K
    products (over the classes for a batch row, over the batch rows for a prototype, whose
    share then flows back to its class), whose rounding grows like sqrt(K) u times the
    largest terms, and the two parts of a batch row's gradient in a small class can cancel.
The kernels keep the positive class out of the softmax sum, so a nearly perfectly predicted
row (1 - softmax_y ~ 3e-4 in the single-row case) still gets a gradient accurate relative to
itself."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, grad_tol_ok as _grad_tol_ok, say, workload
from oracle import proto as oproto

pytestmark = pytest.mark.gpu


U = 2.0 ** -24


def grad_tol_ok(got, ref, B, C):
    return _grad_tol_ok(got, ref, rel=1e-5, floor=max(1e-6, 2 * np.sqrt(max(B, C)) * U))


def run(emb, labels, batch, C, tau, through=True, grad=1.0, demb0=None):
    n, d = emb.shape
    pl = sq.api.ProtoLoss(n, d, C, len(batch))
    E, Y, Bt = dev(emb.astype(np.float32)), dev(labels.astype(np.int32)), dev(batch.astype(np.int32))
    loss, rows, P = pl.forward(E, Y, Bt, tau=tau, row_loss=True, protos=True)
    loss = loss.item()
    g = torch.tensor([grad], dtype=torch.float32, device="cuda")
    demb = None if demb0 is None else dev(demb0.astype(np.float32))
    dE = pl.backward(E, Y, Bt, tau=tau, grad_loss=g, through_prototypes=through, demb=demb)
    torch.cuda.synchronize()
    return loss, rows.cpu().numpy(), P.cpu().numpy(), dE.cpu().numpy()


def row_floor(emb, Pref, tau):
    d = emb.shape[1]
    return 4 * np.sqrt(d) * U * np.linalg.norm(emb, axis=1).max() * np.linalg.norm(Pref, axis=1).max() / tau


def check_forward(emb, labels, batch, C, tau, loss, rows, P):
    Pref, _ = oproto.prototypes(emb, labels, C)
    assert np.abs(P - Pref).max() <= 1e-6 * max(1.0, np.abs(Pref).max())
    L, rref, _ = oproto.loss(emb, labels, batch, C, tau=tau, return_rows=True)
    floor = row_floor(emb, Pref, tau)
    assert np.all(np.abs(rows - rref) <= 1e-5 * np.abs(rref) + floor), np.abs(rows - rref).max()
    assert abs(loss - L) <= 1e-5 * abs(L) + floor * len(batch), (loss, L)


def small_case(d, seed, B=300, scale=True):
    rep = synth.tiny(n_families=60, fam_size=8, seed=seed)
    emb = synth.embeddings(rep.seqs, rep.lens, d).astype(np.float64)
    rng = np.random.default_rng(seed)
    if scale:
        emb *= rng.uniform(0.5, 2.0, (rep.n, 1))
    emb = emb.astype(np.float32)
    labels = rep.family.astype(np.int64).copy()
    labels[labels >= 5] += 1                  # class 5 empty
    C = int(labels.max()) + 3                 # two more empty classes at the end; C not a multiple of 32
    batch = rng.integers(0, rep.n, B)         # repeats allowed; B not a multiple of 32
    return emb, labels, batch, C


@pytest.mark.parametrize("d", [32, 64, 128])
@pytest.mark.parametrize("through", [True, False])
def test_small(d, through):
    emb, labels, batch, C = small_case(d, seed=d)
    tau = 0.1 if through else 0.5
    say(f"proto d={d} C={C} B={len(batch)} through={through}")
    loss, rows, P, dE = run(emb, labels, batch, C, tau, through=through, grad=1.3)
    check_forward(emb, labels, batch, C, tau, loss, rows, P)
    ref = oproto.backward(emb, labels, batch, C, tau=tau, grad_loss=1.3, through_prototypes=through)
    ok, rel = grad_tol_ok(dE, ref, len(batch), C)
    assert ok, rel


def test_edges():
    emb, labels, batch, C = small_case(64, seed=3, B=40)
    n = emb.shape[0]
    say("proto empty batch")
    loss, rows, P, dE = run(emb, labels, batch[:0], C, 0.1)
    assert loss == 0.0 and rows.shape == (0,) and not dE.any()
    say("proto one class")
    one = np.zeros_like(labels)
    loss, rows, P, dE = run(emb, one, batch, 1, 0.1)
    assert abs(loss) <= 1e-6 * len(batch) and np.abs(dE).max() <= 1e-5
    say("proto single row batch")
    loss, rows, P, dE = run(emb, labels, batch[:1], C, 0.1)
    check_forward(emb, labels, batch[:1], C, 0.1, loss, rows, P)
    ok, rel = grad_tol_ok(dE, oproto.backward(emb, labels, batch[:1], C, tau=0.1), 1, C)
    assert ok, rel
    # unlabelled rows (labels -1 and C) and batch entries outside [0, n) contribute nothing
    say("proto unlabelled rows and invalid batch entries")
    lab2 = labels.copy()
    lab2[n - 7:n - 4] = -1
    lab2[n - 4:] = C
    keep = np.arange(n - 7)
    b2 = np.concatenate([batch, [-1, n + 3, n - 1, n - 6]])
    loss, rows, P, dE = run(emb, lab2, b2, C, 0.1, grad=0.7)
    bk = batch                                 # the labelled, in-range part of b2
    L, rref, _ = oproto.loss(emb[keep], lab2[keep], bk, C, tau=0.1, return_rows=True)
    fl = row_floor(emb[keep], oproto.prototypes(emb[keep], lab2[keep], C)[0], 0.1)
    assert abs(loss - L) <= 1e-5 * abs(L) + fl * len(bk)
    assert np.allclose(rows[:len(bk)], rref, rtol=1e-5, atol=fl) and not rows[len(bk):].any()
    ref = oproto.backward(emb[keep], lab2[keep], bk, C, tau=0.1, grad_loss=0.7)
    ok, rel = grad_tol_ok(dE[keep], ref, len(bk), C)
    assert ok, rel
    assert not dE[n - 7:].any()
    # the backward accumulates
    say("proto accumulate")
    base = np.random.default_rng(1).standard_normal(emb.shape).astype(np.float32)
    _, _, _, dE1 = run(emb, labels, batch, C, 0.1)
    _, _, _, dE2 = run(emb, labels, batch, C, 0.1, demb0=base)
    assert np.allclose(dE2 - base, dE1, rtol=1e-5, atol=1e-6)


def test_zipf100k_8192_rows():
    """100,000 sequences in 10,000 rank-Zipf families, d = 128, a batch of 8,192 distinct
    rows; the whole gradient (through the prototypes) against the oracle."""
    rep = workload("zipf100k")
    emb = synth.embeddings(rep.seqs, rep.lens, 128)
    labels = rep.family.astype(np.int64)
    C = int(labels.max()) + 1
    batch = synth.sample_rows(rep.n, 8192, seed=77)
    say(f"proto zipf100k C={C} B=8192")
    loss, rows, P, dE = run(emb, labels, batch, C, 0.1, grad=1.0)
    check_forward(emb, labels, batch, C, 0.1, loss, rows, P)
    ok, rel = grad_tol_ok(dE, oproto.backward(emb, labels, batch, C, tau=0.1), len(batch), C)
    assert ok, rel


def test_rep1m_full_size():
    """1,000,000 sequences, 100,000 families, d = 128, a batch of 65,536 rows: the size the
    benchmark times.  Checked: every prototype; the loss and (prototypes held constant) the
    gradient of 64 sampled batch rows, each of which the oracle computes on its own; with the
    route through the prototypes, the property that the rows of one class receive one and
    the same extra vector, whose class-size-weighted sum is zero (sum_c (softmax - onehot) = 0)."""
    rep = workload("rep1m")
    emb = synth.embeddings(rep.seqs, rep.lens, 128)
    labels = rep.family.astype(np.int64)
    C = int(labels.max()) + 1
    batch = synth.sample_rows(rep.n, 65536, seed=78)
    say(f"proto rep1m n={rep.n} C={C} B=65536")
    loss, rows, P, dE0 = run(emb, labels, batch, C, 0.1, through=False)
    Pref, counts = oproto.prototypes(emb, labels, C)
    assert np.abs(P - Pref).max() <= 1e-6 * max(1.0, np.abs(Pref).max())
    pick = np.sort(np.random.default_rng(5).choice(len(batch), 64, replace=False))
    L, rref, _ = oproto.loss(emb, labels, batch[pick], C, tau=0.1, return_rows=True)
    assert np.all(np.abs(rows[pick] - rref) <= 1e-5 * np.abs(rref) + row_floor(emb, Pref, 0.1))
    ref = oproto.backward(emb, labels, batch[pick], C, tau=0.1, through_prototypes=False)
    ok, rel = grad_tol_ok(dE0[batch[pick]], ref[batch[pick]], len(batch), C)
    assert ok, rel
    assert rows.min() >= -2e-6 and np.isfinite(loss)
    say("proto rep1m through the prototypes")
    _, _, _, dE1 = run(emb, labels, batch, C, 0.1, through=True)
    route = dE1.astype(np.float64) - dE0
    scale = np.abs(route).max()
    for c in np.random.default_rng(6).choice(C, 50, replace=False):
        members = np.nonzero(labels == c)[0]
        others = np.setdiff1d(members, batch)  # rows outside the batch get the route only
        if len(others) > 1:
            assert np.abs(route[others] - route[others[0]]).max() <= 1e-6 * scale
    outside = np.setdiff1d(np.arange(rep.n), batch)
    assert not dE0[outside].any()
    total = route.sum(axis=0)
    assert np.abs(total).max() <= 1e-4 * np.abs(route).sum(axis=0).max()
