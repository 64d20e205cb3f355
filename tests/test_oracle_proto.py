"""Pins for the prototype-contrastive loss oracle (Eq. (pc), Eq. (proto)): hand-worked values,
constructions with a known answer, invariances, torch float64 autograd of an independently
written forward, and central finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import proto


def _case(seed=0, n=60, d=8, C=7):
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((n, d))
    y = rng.integers(0, C, n)
    y[:C] = np.arange(C)                                  # every class present
    batch = rng.integers(0, n, 25)
    return E, y, batch, C


def test_hand_worked_two_classes():
    # p0 = (1, 0), p1 = (0, 1); x = (1, 0) of class 0: logits (10, 0), loss = log(1 + e^-10)
    E = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    y = np.array([0, 0, 1])
    assert proto.loss(E, y, [0], 2) == pytest.approx(4.539889921686465e-05, rel=1e-12)
    # x = (0, 1) of class 1 as well: same value again
    assert proto.loss(E, y, [0, 2], 2) == pytest.approx(2 * 4.539889921686465e-05, rel=1e-12)


def test_singleton_and_symmetric_classes():
    E = np.array([[3.0, -1.0], [2.0, 2.0], [-2.0, -2.0], [5.0, 5.0]])
    y = np.array([0, 1, 1, 2])
    P, counts = proto.prototypes(E, y, 4)
    assert np.array_equal(P[0], E[0]) and np.array_equal(P[1], [0.0, 0.0]) and np.array_equal(P[2], E[3])
    assert list(counts) == [1, 2, 1, 0] and np.array_equal(P[3], [0.0, 0.0])


def test_prototypes_are_centroids():
    E, y, _, C = _case(1)
    P, _ = proto.prototypes(E, y, C)
    for c in range(C):
        assert np.allclose((E[y == c] - P[c]).sum(axis=0), 0.0, atol=1e-12)
    v = np.arange(E.shape[1], dtype=float)
    P2, _ = proto.prototypes(E + v, y, C)                 # translation equivariance
    assert np.allclose(P2, P + v, atol=1e-12)


def test_one_class_gives_zero():
    E, _, batch, _ = _case(2)
    y = np.zeros(E.shape[0], dtype=np.int64)
    assert proto.loss(E, y, batch, 1) == 0.0
    assert np.abs(proto.backward(E, y, batch, 1)).max() == 0.0


def test_equal_prototypes_give_log_c():
    # class c holds u + v_c and u - v_c, so every prototype is u: each term is log C
    rng = np.random.default_rng(3)
    C, d = 5, 6
    u = rng.standard_normal(d)
    V = rng.standard_normal((C, d))
    E = np.concatenate([u + V, u - V])
    y = np.concatenate([np.arange(C), np.arange(C)])
    batch = np.arange(2 * C)
    assert proto.loss(E, y, batch, C) == pytest.approx(2 * C * math.log(C), rel=1e-12)


def test_empty_classes_change_nothing():
    E, y, batch, C = _case(4)
    assert proto.loss(E, y, batch, C + 5) == pytest.approx(proto.loss(E, y, batch, C), rel=1e-14)
    for through in (True, False):
        a = proto.backward(E, y, batch, C + 5, through_prototypes=through)
        b = proto.backward(E, y, batch, C, through_prototypes=through)
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_invariances():
    E, y, batch, C = _case(5)
    base = proto.loss(E, y, batch, C)
    perm = np.random.default_rng(0).permutation(C)
    assert proto.loss(E, perm[y], batch, C) == pytest.approx(base, rel=1e-13)      # relabelling
    assert proto.loss(2.0 * E, y, batch, C, tau=4 * proto.TAU) == pytest.approx(base, rel=1e-13)  # <2f,2p>/4tau
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((E.shape[1],) * 2))
    assert proto.loss(E @ Q, y, batch, C) == pytest.approx(base, rel=1e-12)        # rotation
    assert proto.loss(E, y, batch, C) >= 0.0


def _torch_loss(E, y, batch, C, tau, through):
    """Independent transcription: prototypes as a one-hot average, log_softmax, NLL sum."""
    yt = torch.as_tensor(y)
    onehot = torch.nn.functional.one_hot(yt, C).double()            # [n, C]
    counts = onehot.sum(0)
    present = counts > 0
    P = (onehot.T @ E) / counts.clamp(min=1)[:, None]
    if not through:
        P = P.detach()
    Z = E[torch.as_tensor(batch)] @ P.T / tau
    Z = Z.masked_fill(~present[None, :], float("-inf"))
    return -torch.log_softmax(Z, dim=1)[torch.arange(len(batch)), yt[torch.as_tensor(batch)]].sum()


@pytest.mark.parametrize("through", [True, False])
def test_against_torch_autograd(through):
    E, y, batch, C = _case(6)
    Et = torch.tensor(E, requires_grad=True)
    L = _torch_loss(Et, y, batch, C + 2, 0.25, through)
    (1.7 * L).backward()
    assert proto.loss(E, y, batch, C + 2, tau=0.25) == pytest.approx(L.item(), rel=1e-13)
    got = proto.backward(E, y, batch, C + 2, tau=0.25, grad_loss=1.7, through_prototypes=through)
    assert np.allclose(got, Et.grad.numpy(), rtol=1e-11, atol=1e-13)


def test_finite_differences():
    E, y, batch, C = _case(7, n=30, d=5, C=4)
    got = proto.backward(E, y, batch, C, tau=0.5)
    h = 1e-6
    for r, k in [(0, 0), (3, 2), (int(batch[0]), 4), (17, 1), (29, 3)]:
        p, m = E.copy(), E.copy()
        p[r, k] += h
        m[r, k] -= h
        fd = (proto.loss(p, y, batch, C, tau=0.5) - proto.loss(m, y, batch, C, tau=0.5)) / (2 * h)
        assert abs(fd - got[r, k]) <= 1e-6 * max(1.0, abs(fd)), (r, k)
