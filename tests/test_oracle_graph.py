"""Pins for the graph oracle: a hand-built example, the loop-based construction, symmetry
and degree identities."""
import numpy as np

from oracle import graph as og


def test_hand_example():
    # pairs (i, j, w): 0-1 0.9, 0-2 0.8, 1-2 0.75, 2-3 0.6 (below tau), 0-3 0.8
    pairs = np.array([[0, 1], [0, 2], [1, 2], [2, 3], [0, 3]])
    w = np.array([0.9, 0.8, 0.75, 0.6, 0.8], np.float32)
    offs, cols, vals = og.topk_graph(pairs, w, 4, 0.7)
    assert offs.tolist() == [0, 3, 5, 7, 8]
    assert cols.tolist() == [1, 2, 3, 0, 2, 0, 1, 0]   # node 0: 0.9 (1), then the 0.8 tie by id
    assert np.allclose(vals, [0.9, 0.8, 0.8, 0.9, 0.75, 0.8, 0.75, 0.8])
    offs, cols, _ = og.topk_graph(pairs, w, 4, 0.7, k=1)
    assert offs.tolist() == [0, 1, 2, 3, 4] and cols.tolist() == [1, 0, 0, 0]


def test_matches_loop_construction():
    rng = np.random.default_rng(1)
    n = 60
    a = rng.integers(0, n, 800)
    b = rng.integers(0, n, 800)
    keep = a != b
    pr = np.sort(np.stack([a[keep], b[keep]], 1), axis=1)
    pr = np.unique(pr, axis=0)
    w = rng.choice(np.float32([0.5, 0.7, 0.71, 0.8, 0.8, 0.9, 1.0]), pr.shape[0])  # many ties
    for k in (0, 1, 3, 10):
        x = og.topk_graph(pr, w, n, 0.7, k)
        y = og.topk_graph_loops(pr, w, n, 0.7, k)
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_untruncated_graph_is_symmetric():
    rng = np.random.default_rng(2)
    n = 40
    pr = np.unique(np.sort(rng.integers(0, n, (300, 2)), axis=1), axis=0)
    pr = pr[pr[:, 0] != pr[:, 1]]
    w = rng.random(pr.shape[0]).astype(np.float32)
    offs, cols, vals = og.topk_graph(pr, w, n, 0.5)
    E = {(u, int(c), float(v)) for u in range(n) for c, v in zip(cols[offs[u]:offs[u + 1]], vals[offs[u]:offs[u + 1]])}
    assert all((c, u, v) in E for (u, c, v) in E)
    assert offs[-1] == 2 * int((w >= np.float32(0.5)).sum())


def test_recall():
    offs = np.array([0, 1, 2, 2])
    cols = np.array([1, 0])
    fam = np.array([0, 0, 1])
    assert og.recall_at_k(offs, cols, fam, 5) == 1.0
