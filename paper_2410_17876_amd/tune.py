"""Autotuner for the fused/batched tile shape.

Times qd_batch_apply (or qd_apply_circuit) on a sample of the workload for each
candidate (tile amplitudes, minimum contiguous run) and keeps the fastest. The
choice depends on the precision (bytes per amplitude, LDS per workgroup) and on
the workload's gate mix (how many gates fit a tile), so results are cached per
(device, precision, workload key) in a JSON file.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

CANDIDATES = {
    "c128": [(2048, 64), (3072, 64), (4096, 64), (4096, 128), (8192, 128)],
    "c64": [(4096, 128), (8192, 128), (8192, 256), (16384, 256)],
}


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def load_cache(path: Optional[str]) -> Dict:
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def tune(run: Callable[[int, int], None], precision: str, key: str, cache_path: Optional[str] = None,
         candidates: Optional[Iterable[Tuple[int, int]]] = None, reps: int = 2) -> dict:
    """Pick (tile_amps, min_run) minimising run(tile, run_len)'s wall time.

    run(tile, min_run) must execute the sample workload once and synchronise.
    Each candidate is run once to warm up, then timed `reps` times (best kept).
    """
    cache = load_cache(cache_path)
    ckey = f"{_device_name()}|{precision}|{key}"
    if ckey in cache:
        return dict(cache[ckey], cached=True)
    timings = {}
    for tile, run_len in (candidates or CANDIDATES[precision]):
        run(tile, run_len)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            run(tile, run_len)
            best = min(best, time.perf_counter() - t0)
        timings[f"{tile}/{run_len}"] = best
    tile, run_len = (int(x) for x in min(timings, key=timings.get).split("/"))
    result = {"tile_amps": tile, "min_run": run_len, "timings_s": timings}
    if cache_path:
        cache[ckey] = result
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(result, cached=False)
