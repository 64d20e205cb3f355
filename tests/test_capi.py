"""The C ABI on the CPU: every declared symbol is exported, and argument validation
returns its status code before anything touches a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "subquad.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(subquad_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2602_17330_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2602_17330_amd import build
        build.build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    from paper_2602_17330_amd import _lib
    names = _declared()
    assert len(names) >= 14
    for nm in names:
        assert hasattr(L, nm), nm
        assert nm in _lib.SIGNATURES, nm
    assert set(_lib.SIGNATURES) == set(names)


def test_version(L):
    assert b"gfx950" in L.subquad_version()


NULL = None
FAKE = 4096  # never dereferenced: validation fails first


def test_minhash_validation(L):
    assert L.subquad_minhash(FAKE, FAKE, 10, 32, 4, 64, 1, FAKE, NULL) == 1
    assert b"k = 3" in L.subquad_last_error()
    assert L.subquad_minhash(FAKE, FAKE, 10, 32, 3, 0, 1, FAKE, NULL) == 1
    assert L.subquad_minhash(FAKE, FAKE, 10, 32, 3, 257, 1, FAKE, NULL) == 1
    assert L.subquad_minhash(FAKE, FAKE, 10, 30, 3, 64, 1, FAKE, NULL) == 1
    assert L.subquad_minhash(NULL, FAKE, 10, 32, 3, 64, 1, FAKE, NULL) == 1
    assert L.subquad_minhash(NULL, NULL, 0, 32, 3, 64, 1, NULL, NULL) == 0
    assert L.subquad_minhash(FAKE, FAKE, -1, 32, 3, 64, 1, FAKE, NULL) == 1


def test_lsh_validation(L):
    n = ctypes.c_int64(0)
    ws = L.subquad_lsh_workspace_bytes(1000, 16, 5000)
    assert ws > 1000 * 16 * 16
    assert L.subquad_lsh_workspace_bytes(1 << 28, 32, 0) == 0      # n*b >= 2^32
    # b*r > M
    assert L.subquad_lsh_candidates(FAKE, 1000, 64, 17, 4, NULL, 1, 4096, ws, FAKE, NULL, 5000,
                                    ctypes.byref(n), NULL) == 1
    # workspace too small
    assert L.subquad_lsh_candidates(FAKE, 1000, 64, 16, 4, NULL, 1, 4096, ws - 1, FAKE, NULL, 5000,
                                    ctypes.byref(n), NULL) == 5
    # misaligned workspace
    assert L.subquad_lsh_candidates(FAKE, 1000, 64, 16, 4, NULL, 1, 4096 + 8, ws, FAKE, NULL, 5000,
                                    ctypes.byref(n), NULL) == 1
    # R > 1 without offsets
    assert L.subquad_lsh_candidates(FAKE, 1000, 64, 16, 4, NULL, 3, 4096, ws, FAKE, NULL, 5000,
                                    ctypes.byref(n), NULL) == 1
    assert L.subquad_lsh_candidates(FAKE, 1000, 64, 16, 4, NULL, 1, 4096, ws, FAKE, NULL, 5000,
                                    NULL, NULL) == 1


def test_align_validation(L):
    assert L.subquad_align_workspace_bytes(100) >= 4 * (100 + 512)
    ws = L.subquad_align_workspace_bytes(100)
    assert L.subquad_align_batch_ws(FAKE, FAKE, 10, 32, FAKE, 100, FAKE, 1, 2, FAKE, FAKE, ws, NULL) == 1
    assert L.subquad_align_batch_ws(FAKE, FAKE, 10, 32, FAKE, 100, FAKE, 1001, 1, FAKE, FAKE, ws, NULL) == 1
    assert L.subquad_align_batch_ws(FAKE, FAKE, 10, 80, FAKE, 100, FAKE, 10, 1, FAKE, FAKE, ws, NULL) == 1
    assert L.subquad_align_batch_ws(FAKE, FAKE, 10, 32, FAKE, 100, FAKE, 10, 1, FAKE, FAKE, ws - 1, NULL) == 5
    assert L.subquad_align_batch_ws(FAKE, FAKE, 10, 32, FAKE, 0, FAKE, 10, 1, FAKE, NULL, 0, NULL) == 0


def test_gate_validation(L):
    args = [FAKE, 10, 128, FAKE, FAKE, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, FAKE]
    assert L.subquad_gate_fwd(*args, 48, FAKE, NULL, NULL) == 1          # H not a multiple of 16
    assert L.subquad_gate_fwd(*args[:2], 130, *args[3:], 64, FAKE, NULL, NULL) == 1  # d % 4
    assert L.subquad_gate_fwd(*args[:-1], NULL, 64, FAKE, NULL, NULL) == 1          # null b2
    assert L.subquad_gate_bwd_workspace_bytes(64, 0, 10) >= 8 * (64 * 6 + 1)
    assert L.subquad_gate_bwd_workspace_bytes(64, 5000, 10) >= 5000 * (4 * 8 + 16)
    assert L.subquad_gate_bwd_workspace_bytes(64, -1, 10) == 0
    assert L.subquad_gate_bwd_workspace_bytes(64, 5, -1) == 0
    ws = L.subquad_gate_bwd_workspace_bytes(64, 5, 10)
    assert L.subquad_gate_bwd(*args, 64, FAKE, FAKE, FAKE, FAKE, FAKE, NULL, 4096, ws - 1, NULL) == 5
    assert L.subquad_gate_bwd(*args, 64, FAKE, NULL, FAKE, FAKE, FAKE, NULL, 4096, ws, NULL) == 1
    m = ctypes.c_float(0.5)
    assert L.subquad_gate_train(*args, 64, FAKE, m, NULL, FAKE, FAKE, FAKE, FAKE, FAKE, NULL, 4096, ws - 1,
                                NULL) == 5
    assert L.subquad_gate_train(*args, 64, FAKE, m, NULL, NULL, FAKE, FAKE, FAKE, FAKE, NULL, 4096, ws,
                                NULL) == 1                                         # null loss
    assert L.subquad_gate_train(*args, 64, NULL, m, NULL, FAKE, FAKE, FAKE, FAKE, FAKE, NULL, 4096, ws,
                                NULL) == 1                                         # null labels


def test_check_seqs_validation(L):
    assert L.subquad_check_seqs(FAKE, FAKE, 10, 32, 0, NULL, NULL) == 1
    assert L.subquad_check_seqs(NULL, NULL, 0, 32, 3, NULL, NULL) == 0


def test_binding_rejects_host_tensors():
    import torch
    import paper_2602_17330_amd as sq
    with pytest.raises(ValueError):
        sq.minhash(torch.zeros((2, 32), dtype=torch.uint8), torch.full((2,), 5, dtype=torch.int32), 64)
    with pytest.raises(ValueError):
        sq.check_subst([[0] * 20] * 19)


def test_knobs(L):
    # the defaults the header documents
    assert [L.subquad_get_knob(k) for k in range(4)] == [2, 16, 64, 512]
    assert L.subquad_set_knob(2, 128) == 0 and L.subquad_get_knob(2) == 128
    assert L.subquad_set_knob(2, 0) == 0 and L.subquad_get_knob(2) == 64
    assert L.subquad_set_knob(3, 100) == 1            # not a multiple of 64
    assert L.subquad_set_knob(9, 1) == 1 and L.subquad_get_knob(9) == -1


def test_proto_validation(L):
    ws = L.subquad_proto_workspace_bytes(100, 64, 10, 50)
    assert ws > 0 and L.subquad_proto_workspace_bytes(100, 64, 0, 50) == 0
    args = [FAKE, 100, 64, FAKE, 10, FAKE, 50, ctypes.c_float(0.1)]
    assert L.subquad_proto_fwd(*args, FAKE, NULL, NULL, 4096, ws - 1, NULL) == 5         # short workspace
    assert L.subquad_proto_fwd(*args[:2], 48, *args[3:], FAKE, NULL, NULL, 4096, ws, NULL) == 1  # d
    assert L.subquad_proto_fwd(*args[:-1], ctypes.c_float(0.0), FAKE, NULL, NULL, 4096, ws, NULL) == 1  # tau
    assert L.subquad_proto_fwd(*args, NULL, NULL, NULL, 4096, ws, NULL) == 1             # null loss
    assert L.subquad_proto_bwd(*args, NULL, 1, NULL, 4096, ws, NULL) == 1                # null demb


def test_contrastive_validation(L):
    ws = L.subquad_contrastive_workspace_bytes()
    assert ws >= 8
    assert L.subquad_contrastive_grad(FAKE, FAKE, 10, FAKE, 10, ctypes.c_float(0.5), FAKE, FAKE, 4096, ws - 1,
                                      NULL) == 5
    assert L.subquad_contrastive_grad(FAKE, NULL, 10, FAKE, 10, ctypes.c_float(0.5), FAKE, FAKE, 4096, ws,
                                      NULL) == 1
    assert L.subquad_contrastive_grad(FAKE, FAKE, -1, FAKE, 10, ctypes.c_float(0.5), FAKE, FAKE, 4096, ws,
                                      NULL) == 1
