"""Autotuner of the batched (ensemble) stage launch.

For a given ensemble it times every available tile variant of the persistent
2-D stage kernel and a few persistent-grid sizes with hipEvents on the current
stream, on copies of the member states, and keeps the fastest. Results are
cached in a JSON file (``SNAP_TUNE_CACHE``, default
``~/.cache/snap_tune.json``) keyed by device, element type, tracer count and
the multiset of member sizes.
"""
from __future__ import annotations

import json
import os
from typing import Sequence

import torch

from . import (SNAP_F32, SNAP_F64, DeviceGrid, batched_workspace, snap_batched_tile_variant,
               snap_rk3_step_batched)

MAX_VARIANTS = 6


def _cache_path() -> str:
    return os.environ.get("SNAP_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "snap_tune.json")


def _key(grids: Sequence[DeviceGrid]) -> str:
    g0 = grids[0]
    sizes = sorted((g.nx, g.nz) for g in grids)
    dev = torch.cuda.get_device_name(g0.device)
    dt = "f64" if g0.dtype == torch.float64 else "f32"
    return f"{dev}|{dt}|nt{g0.ntracer}|{sizes}"


def _load() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def candidates(grids: Sequence[DeviceGrid]):
    g0 = grids[0]
    dtype = SNAP_F64 if g0.dtype == torch.float64 else SNAP_F32
    out = []
    for v in range(MAX_VARIANTS):
        shape = snap_batched_tile_variant(dtype, g0.ntracer, v)
        if shape is not None and (v == 0 or g0.ntracer == 0):
            out.append((v, shape))
    return out


def time_config(grids, qs, dts, work, variant: int, nblocks: int, repeats: int = 3) -> float:
    """Median milliseconds of one batched RK3 step (states are advanced)."""
    snap_rk3_step_batched(grids, qs, dts, work, variant, nblocks)   # warm-up
    times = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        snap_rk3_step_batched(grids, qs, dts, work, variant, nblocks)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return sorted(times)[len(times) // 2]


def tune_batched(grids: Sequence[DeviceGrid], qs: Sequence[torch.Tensor], dts: Sequence[float],
                 repeats: int = 3, use_cache: bool = True) -> dict:
    """Fastest (variant, nblocks) for this ensemble; the given states are not modified."""
    key = _key(grids)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return db[key]
    copies = [q.clone() for q in qs]
    work = batched_workspace(grids)
    cus = torch.cuda.get_device_properties(grids[0].device).multi_processor_count
    trials = []
    for v, shape in candidates(grids):
        for nb in (0, cus, 2 * cus, 4 * cus):
            ms = time_config(grids, copies, dts, work, v, nb, repeats)
            trials.append({"variant": v, "tile": list(shape), "nblocks": nb, "ms": ms})
    best = min(trials, key=lambda t: t["ms"])
    result = {"variant": best["variant"], "tile": best["tile"], "nblocks": best["nblocks"],
              "ms": best["ms"], "trials": trials}
    if use_cache:
        db[key] = result
        _store(db)
    return result
