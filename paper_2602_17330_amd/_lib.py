"""ctypes loader for libsubquad.so (the C ABI declared in include/subquad.h)."""
from __future__ import annotations

import ctypes
import functools
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsubquad.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_RESIDUE", 3: "ERR_LENGTH", 4: "ERR_CAPACITY",
          5: "ERR_WORKSPACE", 6: "ERR_HIP"}
OK, ERR_ARG, ERR_RESIDUE, ERR_LENGTH, ERR_CAPACITY, ERR_WORKSPACE, ERR_HIP = range(7)

c_i32, c_i64, c_u64, c_sz, c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "subquad_last_error": (ctypes.c_char_p, []),
    "subquad_version": (ctypes.c_char_p, []),
    "subquad_set_knob": (ctypes.c_int, [c_i32, c_i32]),
    "subquad_get_knob": (c_i32, [c_i32]),
    "subquad_profile_enable": (ctypes.c_int, [c_i32]),
    "subquad_profile_only": (ctypes.c_int, [ctypes.c_char_p]),
    "subquad_profile_report": (c_i64, [ctypes.c_char_p, c_sz]),
    "subquad_check_seqs": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_i32, c_p, c_p]),
    "subquad_minhash": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_i32, c_i32, c_u64, c_p, c_p]),
    "subquad_lsh_workspace_bytes": (c_sz, [c_i64, c_i32, c_i64]),
    "subquad_lsh_candidates": (ctypes.c_int, [c_p, c_i64, c_i32, c_i32, c_i32, c_p, c_i64, c_p, c_sz,
                                              c_p, c_p, c_i64, c_p, c_p]),
    "subquad_lsh_candidates_async": (ctypes.c_int, [c_p, c_i64, c_i32, c_i32, c_i32, c_p, c_i64, c_p,
                                                    c_sz, c_p, c_p, c_i64, c_p, c_p, c_p]),
    "subquad_self_scores": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_p, c_p]),
    "subquad_align_batch": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i32, c_i32,
                                           c_p, c_p]),
    "subquad_align_workspace_bytes": (c_sz, [c_i64]),
    "subquad_align_batch_ws": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i32, c_i32,
                                              c_p, c_p, c_sz, c_p]),
    "subquad_align_batch_dev": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_i64, c_p, c_p, c_i32, c_i32,
                                               c_p, c_p, c_sz, c_p]),
    "subquad_align_batch_noalloc": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i32, c_i32,
                                                   c_p, c_p]),
    "subquad_gate_fwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p,
                                        c_p, c_p, c_i32, c_p, c_p, c_p]),
    "subquad_gate_bwd_workspace_bytes": (c_sz, [c_i32, c_i64, c_i64]),
    "subquad_gate_train": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_p, c_p, c_i32,
                                          c_p, ctypes.c_float, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "subquad_gate_train_set": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_p, c_p,
                                              c_i32, c_p, ctypes.c_float, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz,
                                              c_p]),
    "subquad_gate_train_set_dev": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_p,
                                                  c_p, c_p, c_i32, c_p, ctypes.c_float, c_p, c_p, c_p, c_p, c_p, c_p,
                                                  c_p, c_p, c_sz, c_p]),
    "subquad_gate_bwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p,
                                        c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "subquad_edit_cost_matrix": (ctypes.c_int, [c_p, c_p]),
    "subquad_edit_batch_ws": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i32, c_p, c_p, c_sz,
                                             c_p]),
    "subquad_gate3_fwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p,
                                         c_p, c_p, c_i32, c_p, c_p, c_p]),
    "subquad_gate3_bwd_workspace_bytes": (c_sz, [c_i32]),
    "subquad_gate3_bwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p,
                                         c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "subquad_graph_workspace_bytes": (c_sz, [c_i64, c_i64]),
    "subquad_graph_topk": (ctypes.c_int, [c_p, c_p, c_i64, c_i64, ctypes.c_float, c_i32, c_p, c_sz, c_p, c_p,
                                          c_p, c_i64, c_p, c_p]),
    "subquad_contrastive_workspace_bytes": (c_sz, []),
    "subquad_contrastive_grad": (ctypes.c_int, [c_p, c_p, c_i64, c_p, c_i64, ctypes.c_float, c_p, c_p, c_p, c_sz,
                                                c_p]),
    "subquad_rmt_workspace_bytes": (c_sz, [c_i64, c_i32]),
    "subquad_rmt_threshold": (ctypes.c_int, [c_p, c_p, c_p, c_i64, c_i64, c_i32, c_i32, c_u64, c_p, c_p, c_p, c_p,
                                             c_sz, c_p]),
    "subquad_rmt_lambda_max": (ctypes.c_int, [c_p, c_p, c_p, c_i64, c_i64, ctypes.c_double, c_i32, c_u64, c_p, c_p,
                                              c_sz, c_p]),
    "subquad_proto_workspace_bytes": (c_sz, [c_i64, c_i32, c_i64, c_i64]),
    "subquad_proto_fwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i64, ctypes.c_float, c_p, c_p,
                                         c_p, c_p, c_sz, c_p]),
    "subquad_proto_bwd": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_i64, c_p, c_i64, ctypes.c_float, c_p, c_i32,
                                         c_p, c_p, c_sz, c_p]),
}


KNOBS = {"minhash_blocks_per_cu": 0, "align_blocks_per_cu": 1, "gate_groups_per_cu": 2,
         "emit_threads": 3}


class SubquadError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


@functools.lru_cache(maxsize=1)
def lib() -> ctypes.CDLL:
    """Load the built library; raises if it has not been built (no fallback exists)."""
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2602_17330_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def check(status: int) -> None:
    if status != OK:
        raise SubquadError(status, lib().subquad_last_error().decode())


def profile_enable(on: bool = True) -> None:
    check(lib().subquad_profile_enable(1 if on else 0))


def profile_only(name: str | None = None) -> None:
    """Time only the launches of kernel `name` while timing is on (None: every kernel)."""
    check(lib().subquad_profile_only(name.encode() if name else None))


def profile_report() -> dict:
    """{kernel name: (launches, total ms)} of the launches timed since profile_enable."""
    need = lib().subquad_profile_report(None, 0)
    buf = ctypes.create_string_buffer(int(need) + 1)
    lib().subquad_profile_report(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out
