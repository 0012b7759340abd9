"""Autotuner for the ORCA step: picks the grid cell size (as a fraction of
the neighbour distance) and, for batches, the launch form of the step kernel
(persistent with per-XCD tile queues, or one workgroup per tile), the lanes
per workgroup and the compiled neighbour-list capacity, by timing real steps
on the caller's state.

Results are cached in a JSON file keyed by device architecture, form, agent
count bucket (powers of two), density bucket (half-octaves of agents/m^2) and
neighbour cap; the cache path is $ORCA_AUTOTUNE_CACHE or
~/.cache/orca_mi355x/autotune.json.  Timing uses HIP events on the current
stream; the caller's state is never modified (steps write to a scratch copy).
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import orca

FACTORS = (1.0, 0.5, 1.0 / 3.0, 0.25, 0.2)
MODES = (0, 1)


def cache_path() -> str:
    return os.environ.get("ORCA_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "orca_mi355x",
                                       "autotune.json"))


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    path = cache_path()
    data = _load()
    data[key] = value
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover - CPU-only environments
        return "unknown"


def _density(state: orca.State) -> float:
    x0, x1 = float(state.px.min()), float(state.px.max())
    y0, y1 = float(state.py.min()), float(state.py.max())
    area = max((x1 - x0) * (y1 - y0), 1.0)
    return state.n / area


def cache_key(form: str, n: int, density: float, k: int) -> str:
    nb = int(round(math.log2(max(n, 1))))
    db = round(2.0 * math.log2(max(density, 1e-6))) / 2.0
    return f"{_arch()}|{form}|n2^{nb}|d2^{db}|k{k}"


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def tune_plain(state: orca.State, params, ws: orca.Workspace,
               factors: Sequence[float] = FACTORS, reps: int = 5,
               use_cache: bool = True) -> dict:
    """Best cell size for orca_step on this state.  Returns
    {"cell_size": cs, "factor": f, "ms": t, "timings": {f: t}}."""
    key = cache_key("plain", state.n, _density(state), int(params.max_neighbors))
    if use_cache:
        hit = _load().get(key)
        if hit is not None:
            return dict(hit, cell_size=hit["factor"] * params.neighbor_dist, cached=True)
    out = state.clone()
    timings = {}
    for f in factors:
        p = dataclasses.replace(params, cell_size=f * params.neighbor_dist)
        timings[f] = _time_ms(lambda: orca.step(state, p, ws, out=out), reps)
    best = min(timings, key=timings.get)
    res = {"factor": best, "ms": timings[best],
           "timings": {str(k): v for k, v in timings.items()}}
    _store(key, res)
    return dict(res, cell_size=best * params.neighbor_dist, cached=False)


BLOCKS = (64, 128, 256)
K_TILES = (4, 8, 10, 12, 16, 20, 24, 32)  # neighbour capacities compiled into the kernels


def tune_batched(state: orca.State, scene_off, scene_params: List, ws: orca.Workspace,
                 factors: Sequence[float] = FACTORS, modes: Iterable[int] = MODES,
                 blocks: Sequence[int] = BLOCKS, reps: int = 5,
                 use_cache: bool = True) -> dict:
    """Best (cell-size factor, launch form, lanes per workgroup, neighbour
    tile) for orca_step_batched, by coordinate search in that order, each
    stage timing its candidates with the choices made so far (the tile: the
    smallest compiled capacity holding k and the next two).  Returns
    {"factor", "mode", "block", "k_tile", "ms", "timings", "params" (tuned
    per-scene list)}."""
    k = max(int(p.max_neighbors) for p in scene_params)
    key = cache_key(f"batched{len(scene_params)}", state.n, _density(state), k)
    hit = _load().get(key) if use_cache else None
    if hit is None:
        out = state.clone()
        timings = {}

        def run(f, m, b, kt):
            prm = [dataclasses.replace(p, cell_size=f * p.neighbor_dist) for p in scene_params]
            batch = orca.Batch(scene_off, prm, mode=m, block=b, k_tile=kt)
            t = _time_ms(lambda: orca.step_batched(state, batch, ws, out=out), reps)
            timings[f"{f:.4f}/{m}/{b}/{kt}"] = t
            return t

        best = {"factor": factors[0], "mode": 0, "block": 128, "k_tile": 0}
        f = min(factors, key=lambda f: run(f, best["mode"], best["block"], best["k_tile"]))
        best["factor"] = f
        best["mode"] = min(modes, key=lambda m: run(f, m, best["block"], best["k_tile"]))
        best["block"] = min(blocks, key=lambda b: run(f, best["mode"], b, best["k_tile"]))
        tiles = [t for t in K_TILES if t >= k][:3]
        best["k_tile"] = min(tiles, key=lambda kt: run(f, best["mode"], best["block"], kt))
        best["ms"] = timings[f"{f:.4f}/{best['mode']}/{best['block']}/{best['k_tile']}"]
        hit = dict(best, timings=timings)
        _store(key, hit)
        cached = False
    else:
        cached = True
    prm = [dataclasses.replace(p, cell_size=hit["factor"] * p.neighbor_dist)
           for p in scene_params]
    return dict(hit, params=prm, cached=cached)
