"""Autotuner for the launch-shape knobs of libsubquad.

Knobs only choose grid/block shapes (persistent blocks per CU, pair groups per CU, the run
scan's block size); they never change a result, so tuning is a pure timing search.  Each
knob is searched over a short candidate list on the caller's own workload (a ``Pipeline``),
timing its stage with HIP events, and the best values are cached in a JSON file keyed by
GPU architecture and workload size bucket.
"""
from __future__ import annotations

import json
import math
import os

import torch

from ._lib import KNOBS, check, lib

CANDIDATES = {
    "minhash_blocks_per_cu": [1, 2],
    "align_blocks_per_cu": [4, 8, 16],
    "gate_groups_per_cu": [16, 32, 64, 128, 256],
    "emit_threads": [256, 512, 1024],
}
STAGE_OF = {"minhash_blocks_per_cu": "minhash", "align_blocks_per_cu": "align",
            "gate_groups_per_cu": "gate", "emit_threads": "lsh"}


def set_knob(name: str, value: int) -> None:
    check(lib().subquad_set_knob(KNOBS[name], int(value)))


def get_knob(name: str) -> int:
    return int(lib().subquad_get_knob(KNOBS[name]))


def _time(fn, reps: int) -> float:
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    fn()  # warm
    ts = []
    for _ in range(reps):
        ev[0].record()
        fn()
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    ts.sort()
    return ts[len(ts) // 2]


def _key(pipe) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    nb = int(math.log2(max(pipe.n, 1)))
    pb = int(math.log2(max(pipe.P, 1)))
    return f"{arch}/n2^{nb}/P2^{pb}/M{pipe.cfg.M}/b{pipe.cfg.b}"


def tune(pipe, reps: int = 3, cache_path: str | None = None, knobs=None) -> dict:
    """Search every knob on ``pipe`` (after a first ``pipe.step()``); apply and return the
    best values. Reads/writes ``cache_path`` when given."""
    key = _key(pipe)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            for name, v in cache[key]["best"].items():
                set_knob(name, v)
            return cache[key]
    stage_fn = {
        "minhash": pipe.minhash,
        "lsh": pipe.lsh,
        "align": pipe.align,
        "gate": pipe.gate,
    }
    best, timings = {}, {}
    for name in knobs or CANDIDATES:
        fn = stage_fn[STAGE_OF[name]]
        res = {}
        for v in CANDIDATES[name]:
            set_knob(name, v)
            res[v] = _time(fn, reps)
        b = min(res, key=res.get)
        set_knob(name, b)
        best[name] = b
        timings[name] = {str(k): v for k, v in res.items()}
    entry = {"best": best, "ms": timings}
    if cache_path:
        cache[key] = entry
        tmp = cache_path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return entry


def reset() -> None:
    for name in KNOBS:
        set_knob(name, 0)
