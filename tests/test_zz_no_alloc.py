"""The allocation-free alignment entry point against the workspace entry point.

subquad_align_batch_noalloc takes its scratch from a fixed device array inside the library.
It is called twice in a row through the C ABI, the second time on a smaller batch, and each
call must give exactly the scores of subquad_align_batch_ws (and of the oracle) on the same
pairs; the second call must not see anything the first one left in the shared array.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2602_17330_amd as sq
import synth
from helpers import dev, say, sw_oracle
from paper_2602_17330_amd import _lib, api

pytestmark = pytest.mark.gpu


def _inputs(n, P, seed, stride=32):
    rng = np.random.default_rng(seed)
    lens = rng.integers(3, stride + 1, n).astype(np.int32)
    seqs = np.full((n, stride), synth.PAD, np.uint8)
    for i in range(n):
        seqs[i, : lens[i]] = rng.integers(0, 20, lens[i])
    pairs = np.stack([rng.integers(0, n, P), rng.integers(0, n, P)], 1).astype(np.int32)
    return seqs, lens, pairs


def _noalloc(seqs_t, lens_t, pairs_t, S_t, go, ge):
    out = torch.full((pairs_t.shape[0],), -7, dtype=torch.int32, device="cuda")
    st = _lib.lib().subquad_align_batch_noalloc(
        seqs_t.data_ptr(), lens_t.data_ptr(), seqs_t.shape[0], seqs_t.shape[1], pairs_t.data_ptr(),
        pairs_t.shape[0], S_t.data_ptr(), go, ge, out.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    return out


def _ws(seqs_t, lens_t, pairs_t, S_t, go, ge):
    out = torch.empty(pairs_t.shape[0], dtype=torch.int32, device="cuda")
    P = pairs_t.shape[0]
    nb = int(_lib.lib().subquad_align_workspace_bytes(P))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st = _lib.lib().subquad_align_batch_ws(
        seqs_t.data_ptr(), lens_t.data_ptr(), seqs_t.shape[0], seqs_t.shape[1], pairs_t.data_ptr(), P,
        S_t.data_ptr(), go, ge, out.data_ptr(), ws.data_ptr(), nb,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    return out


def test_noalloc_two_calls_match_workspace_entry(blosum62):
    S_t = dev(blosum62)
    # first call: the largest batch the array takes; second call: a smaller one (other lengths)
    for P, n, seed, stride, (go, ge) in ((api.ALIGN_NOALLOC_MAX_PAIRS, 20_000, 5, 32, (10, 1)),
                                         (3_001, 700, 6, 64, (11, 2))):
        seqs, lens, pairs = _inputs(n, P, seed, stride)
        seqs_t, lens_t, pairs_t = dev(seqs), dev(lens), dev(pairs)
        say(f"align noalloc P={P} n={n} stride={stride} gaps={go}/{ge}")
        got = _noalloc(seqs_t, lens_t, pairs_t, S_t, go, ge)
        ref = _ws(seqs_t, lens_t, pairs_t, S_t, go, ge)
        torch.cuda.synchronize()
        got, ref = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got, ref), f"P={P}: {(got != ref).sum()} scores differ from the workspace entry"
        k = np.random.default_rng(seed).choice(P, min(P, 20_000), replace=False)
        assert np.array_equal(got[k], sw_oracle(seqs, lens, pairs[k], blosum62, go, ge))


def test_noalloc_rejects_too_many_pairs(blosum62):
    seqs, lens, pairs = _inputs(10, 4, 1)
    S_t = dev(blosum62)
    seqs_t, lens_t = dev(seqs), dev(lens)
    big = torch.zeros((api.ALIGN_NOALLOC_MAX_PAIRS + 1, 2), dtype=torch.int32, device="cuda")
    out = torch.empty(big.shape[0], dtype=torch.int32, device="cuda")
    st = _lib.lib().subquad_align_batch_noalloc(
        seqs_t.data_ptr(), lens_t.data_ptr(), 10, 32, big.data_ptr(), big.shape[0], S_t.data_ptr(), 10, 1,
        out.data_ptr(), None)
    assert st == _lib.ERR_ARG
    assert b"at most" in _lib.lib().subquad_last_error()
    # the binding raises the same error; an empty batch is a no-op
    with pytest.raises(_lib.SubquadError):
        sq.api.align_noalloc(seqs_t, lens_t, big, S_t)
    assert sq.api.align_noalloc(seqs_t, lens_t, big[:0], S_t).numel() == 0
