"""The parity tests' own checks, on the CPU: the widened gradient bound used where a float32
ReLU decision may go either way accepts every mix of those decisions and nothing more; the
chunked oracle backward equals the one-call backward."""
import numpy as np

import synth
from helpers import ambiguous_flip_bounds, gate_backward_chunked, grads_ok_widened
from oracle import gate as ogate
from oracle import sw as osw

NAMES = ("W1", "b1", "w2", "b2", "emb")


def _case(P=300, seed=3):
    rep = synth.tiny(n_families=30, fam_size=6, seed=seed)
    S = synth.load_blosum62()
    pairs = synth.random_pairs(rep.n, P, seed, family=rep.family).astype(np.int64)
    W1, b1, w2, b2 = [np.asarray(w, np.float64) for w in synth.gate_params(16, seed=seed)]
    oa = dict(emb=synth.embeddings(rep.seqs, rep.lens, 32), lens=rep.lens, vgene=rep.vgene,
              self_scores=osw.self_scores(rep.seqs, rep.lens, S), pairs=pairs,
              align=osw.scores_pairs(rep.seqs, rep.lens, pairs, S), W1=W1, b1=b1.copy(), w2=w2, b2=b2)
    # put hidden unit 5 of pair 7 and unit 9 of pair 40 exactly on the kink
    _, a = ogate.forward(**oa, return_all=True)
    for p, k in ((7, 5), (40, 9)):
        oa["b1"][k] -= a["z"][p, k]
        _, a = ogate.forward(**oa, return_all=True)
    gf = synth.upstream_grad(pairs.shape[0], seed=seed)
    return oa, gf, a


def test_chunked_backward_equals_one_call():
    oa, gf, _ = _case()
    a = ogate.backward(**oa, grad_f=gf)
    b = gate_backward_chunked(oa, gf, chunk=37)
    for k in NAMES + ("f",):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-15)


def test_widened_bound_accepts_flipped_decisions_only():
    oa, gf, a = _case()
    n_amb, ew, nw = ambiguous_flip_bounds(oa, gf)
    assert n_amb >= 2
    ref = ogate.backward(**oa, grad_f=gf)
    # every mix of the two ambiguous decisions passes
    for bits in ((False, False), (True, False), (False, True), (True, True)):
        mask = a["z"] > 0
        mask[7, 5], mask[40, 9] = bits
        alt = ogate.backward(**oa, grad_f=gf, relu_mask=mask)
        for k in NAMES:
            assert grads_ok_widened(alt[k], ref[k], ew[k], nw[k])[0], (bits, k)
    # flipping a decision that is not ambiguous fails
    mask = a["z"] > 0
    big = np.argmax(np.abs(a["z"][3]))
    mask[3, big] = ~mask[3, big]
    alt = ogate.backward(**oa, grad_f=gf, relu_mask=mask)
    assert not all(grads_ok_widened(alt[k], ref[k], ew[k], nw[k])[0] for k in NAMES)
    # a pair left out fails
    drop = dict(oa, pairs=oa["pairs"][1:], align=oa["align"][1:])
    alt = ogate.backward(**drop, grad_f=gf[1:])
    assert not all(grads_ok_widened(alt[k], ref[k], ew[k], nw[k])[0] for k in NAMES)
