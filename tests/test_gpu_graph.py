"""GPU similarity graph (tau threshold + per-node top-k) against the oracle: bit-exact CSR.
Weights are synthetic float32 values with many exact ties, shared by both sides."""
import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, say
from oracle import graph as og

pytestmark = pytest.mark.gpu


def _weights(P, seed):
    rng = np.random.default_rng(seed)
    levels = np.float32([-0.2, 0.3, 0.69999, 0.7, 0.7, 0.75, 0.8, 0.8, 0.95, 1.0])
    w = rng.choice(levels, P).astype(np.float32)
    free = rng.random(P) < 0.3                     # some weights without ties
    w[free] = rng.random(int(free.sum())).astype(np.float32)
    return w


def _check(pairs, w, n, tau, k):
    rows, cols, vals = sq.graph_topk(dev(pairs.astype(np.int32)), dev(w), n, tau, k)
    torch.cuda.synchronize()
    ro, co, vo = og.topk_graph(pairs, w, n, tau, k)
    assert np.array_equal(rows.cpu().numpy(), ro)
    assert np.array_equal(cols.cpu().numpy(), co)
    assert np.array_equal(vals.cpu().numpy(), vo)


@pytest.mark.parametrize("k", [0, 1, 5, 100])
def test_small_with_ties(k):
    r = synth.tiny(n_families=40, fam_size=6, seed=21)
    pairs = synth.random_pairs(r.n, 4000, 3, family=r.family)
    w = _weights(pairs.shape[0], 1)
    say(f"graph small k={k}")
    _check(pairs, w, r.n, 0.7, k)


def test_hub_and_edges():
    n = 3000
    pairs = np.stack([np.zeros(n - 1, np.int64), np.arange(1, n)], 1)   # node 0 joined to all
    w = _weights(pairs.shape[0], 2)
    say("graph hub")
    for k in (0, 3, 64):
        _check(pairs, w, n, 0.7, k)
    _check(pairs, np.full(pairs.shape[0], 0.1, np.float32), n, 0.7, 0)   # nothing passes
    _check(np.zeros((0, 2), np.int64), np.zeros(0, np.float32), n, 0.7, 5)  # no pairs


def test_million_nodes():
    n = 1_000_000
    pairs = synth.random_pairs(n, 3_000_000, 4)
    w = _weights(pairs.shape[0], 3)
    say("graph 1M nodes 3M pairs")
    _check(pairs, w, n, 0.7, 10)
