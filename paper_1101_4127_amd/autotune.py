"""Autotuner of the march's launch parameters on a given workload.

The parameters change the schedule, never the result (packet histories and
deposits are the same for every choice; the GPU parity tests check this):

* march kind: tiled (8^3 tiles, packets handed from tile to tile) or
  per-packet;
* tiled march: packets per run of a tile (run_len), lanes that must be free
  before a wavefront refills (refill_min), blocks per compute unit;
* per-packet march: brick side of the cell layout (brick_log2), packet ids a
  wavefront claims at once (wave_chunk), refill_min, blocks per compute unit.

The search is coordinate descent from the library's defaults: one parameter
at a time over its candidates, the others held, keeping the fastest; two
sweeps.  A candidate is timed as the median march time (HIP events around the
march of every sub-step, RT_TIME_MARCH) of a few steps after a warm-up step
on the workload itself.  Results are cached in a JSON file keyed by the
workload's shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
from typing import Callable, Dict, List, Optional, Tuple

SPACE_TILED: Dict[str, List[int]] = {
    "run_len": [1024, 2048, 4096, 8192],
    "refill_min": [8, 16, 24, 32],
    "blocks_per_cu": [0, 2, 3],
}
SPACE_DIRECT: Dict[str, List[int]] = {
    "brick_log2": [0, 1, 2, 3],
    "wave_chunk": [64, 256, 1024],
    "refill_min": [4, 8, 16],
    "blocks_per_cu": [0, 2, 4],
}
DEFAULT_TILED = {"direct": False, "run_len": 0, "refill_min": 0, "blocks_per_cu": 0}
DEFAULT_DIRECT = {"direct": True, "brick_log2": -1, "wave_chunk": 0, "refill_min": 0, "blocks_per_cu": 0}


def signature(work, fp64: bool) -> str:
    """Key of a workload's shape: what the best schedule depends on."""
    key = dict(n=list(map(int, work.n)), bins=int(work.bins.n_bins), y_he=float(work.y_he) > 0.0,
               thermal=not bool(work.flags & 0x1), fp64=bool(fp64), packets=int(work.packets),
               n_sub=int(work.n_sub), sources=int(len(work.src_ndot)), name=str(work.name))
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:16]


def coordinate_descent(measure: Callable[[dict], float], start: dict, space: Dict[str, List[int]],
                       sweeps: int = 2) -> Tuple[dict, float, List[Tuple[dict, float]]]:
    """Minimise measure(config) one coordinate at a time; returns the best
    config, its time and every (config, time) measured."""
    seen: Dict[str, float] = {}
    log: List[Tuple[dict, float]] = []

    def cost(cfg: dict) -> float:
        k = json.dumps(cfg, sort_keys=True)
        if k not in seen:
            seen[k] = float(measure(dict(cfg)))
            log.append((dict(cfg), seen[k]))
        return seen[k]

    best = dict(start)
    best_t = cost(best)
    for _ in range(sweeps):
        changed = False
        for name, values in space.items():
            for v in values:
                if best.get(name) == v:
                    continue
                cand = dict(best)
                cand[name] = v
                t = cost(cand)
                if t < best_t:
                    best, best_t, changed = cand, t, True
        if not changed:
            break
    return best, best_t, log


def march_time(work, cfg: dict, *, fp64: bool, steps: int = 2, seed0: int = 100) -> float:
    """Median march time (ms per step) of the workload under cfg."""
    import torch
    from . import rt
    kw = dict(cfg)
    if not kw.get("direct"):
        kw["inflight"] = -(-int(work.packets) // int(work.n_sub))
    s = rt.Solve(work, fp64=fp64, time_march=True, **kw)
    try:
        s.step(seed=seed0)                       # warm-up
        times = []
        for i in range(steps):
            st = s.step(seed=seed0 + 1 + i)
            times.append(st["march_ms"])
        torch.cuda.synchronize()
    finally:
        s.release()
    return statistics.median(times)


def tune(work, *, fp64: bool = False, kinds=("tiled", "direct"), steps: int = 2, sweeps: int = 2,
         cache: Optional[str] = None, measure: Optional[Callable[[dict], float]] = None) -> dict:
    """Best launch parameters for work; measure(cfg) -> ms overrides the GPU
    timing (tests).  Returns {"config", "march_ms", "trials", "signature"}."""
    sig = signature(work, fp64)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if sig in table:
            return table[sig]
    if measure is None:
        def measure(cfg):
            return march_time(work, cfg, fp64=fp64, steps=steps)
    best, best_t, trials = None, float("inf"), []
    for kind in kinds:
        start, space = (DEFAULT_TILED, SPACE_TILED) if kind == "tiled" else (DEFAULT_DIRECT, SPACE_DIRECT)
        cfg, t, log = coordinate_descent(measure, start, space, sweeps=sweeps)
        trials += log
        if t < best_t:
            best, best_t = cfg, t
    result = {"config": best, "march_ms": best_t, "trials": [[c, t] for c, t in trials], "signature": sig}
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[sig] = result
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return result
