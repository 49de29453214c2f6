"""Launch-shape autotuner for the FDTD kernels, with a JSON cache.

For one grid it times every candidate (kernel variant, TY, TZ) on the GPU
with the library's own event timing of the update kernels, keeps the fastest
and caches it under a key made of the device name, grid size, CPML
thickness and precision.  For a batch it does the same over the batched
tile shapes (TX, TY) and TZ.  Every variant computes bitwise the same fields
(the per-element arithmetic is shared), so tuning never changes results.

The cache file is ``$FDTD_TUNE_CACHE`` if set, else
``~/.cache/mi355fdtd/tune.json``.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, List, Sequence, Tuple

from . import fdtd

# (variant, TY, TZ): the split pass; fused tiles 64 x TY; two-step tiles
# 60 x TY in 64 x (TY + 4) regions.
GRID_CANDIDATES: List[Tuple[int, int, int]] = (
    [(fdtd.KERNEL_SPLIT, 0, 0)]
    + [(fdtd.KERNEL_FUSED, ty, tz) for ty in (4, 8) for tz in (16, 24, 32, 48, 64)]
    + [(fdtd.KERNEL_TB2, 8, tz) for tz in (16, 18, 20, 22, 24, 28, 32, 40)]
    + [(fdtd.KERNEL_TB2, 4, tz) for tz in (16, 20, 28)]
    + [(fdtd.KERNEL_TB2, 12, tz) for tz in (16, 20, 24)]
)
# Grids with Debye media take the split pass or the fused pass (8-row tiles;
# TZ-plane chunks of the CPML tile groups).  Their cache key needs its own
# suffix (grid_key does not see the poles).
DEBYE_CANDIDATES: List[Tuple[int, int, int]] = (
    [(fdtd.KERNEL_SPLIT, 0, 0)] + [(fdtd.KERNEL_FUSED, 8, tz) for tz in (16, 24, 32, 48, 64)])
# (TX, TY, TZ, persistent): one-step batch tiles, then two-step 60 x 8
# tiles launched per CPML group (0) or as persistent work-queue launches (1).
BATCH_CANDIDATES: List[Tuple[int, int, int, int]] = (
    [(tx, ty, tz, 0) for (tx, ty) in ((32, 8), (32, 16), (64, 8)) for tz in (16, 32, 64)]
    + [(60, 8, tz, p) for tz in (16, 20, 24, 32, 48, 64) for p in (1, 0)]
    + [(60, 8, tz, 1) for tz in (96, 128)])


def tuning_steps(batch: bool = False, warmup: int = 4, steps: int = None) -> int:
    """Steps one tuning pass takes with the default candidates."""
    if batch:
        return len(BATCH_CANDIDATES) * (warmup + (steps or 20))
    return len(GRID_CANDIDATES) * (warmup + (steps or 24))


def cache_path() -> str:
    p = os.environ.get("FDTD_TUNE_CACHE")
    return p or os.path.join(os.path.expanduser("~"), ".cache", "mi355fdtd", "tune.json")


def load_cache(path: str = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, value: dict, path: str = None) -> None:
    path = path or cache_path()
    d = load_cache(path)
    d[key] = value
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def grid_key(params: dict, precision: int = 32, device: str = None) -> str:
    return (f"{device or _device_name()}|grid|{params['nx']}x{params['ny']}x{params['nz']}"
            f"|npml{params.get('npml', 0)}|fp{precision}")


def batch_key(dims: Sequence[Tuple[int, int, int]], npml: int, precision: int = 32, device: str = None) -> str:
    cells = sum(a * b * c for a, b, c in dims)
    # shape class: grid count and total cells to 2 significant digits
    return f"{device or _device_name()}|batch|{len(dims)}|{float(f'{cells:.2g}'):.3g}|npml{npml}|fp{precision}"


def _time_grid(g: "fdtd.Grid", cand, warmup: int, steps: int) -> float:
    g.set_kernel(*cand)
    g.step(warmup)
    g.timing(True)
    g.kernel_time()          # drains and resets
    g.step(steps)
    ms, n = g.kernel_time()
    g.timing(False)
    return ms / max(n, 1)


def tune_grid(make_grid, key: str, candidates: Iterable = None, warmup: int = 4, steps: int = 24,
              path: str = None, force: bool = False, log=None) -> dict:
    """make_grid(max_steps) -> a set-up fdtd.Grid, or a Grid with room for
    tuning_steps() more steps.  Returns the cached or newly measured best
    {variant, tile_y, tile_z, ms_per_step}."""
    cache = load_cache(path)
    if key in cache and not force:
        return cache[key]
    cands = list(candidates or GRID_CANDIDATES)
    g = make_grid if isinstance(make_grid, fdtd.Grid) else make_grid(len(cands) * (warmup + steps) + 4)
    results = []
    for cand in cands:
        ms = _time_grid(g, cand, warmup, steps)
        results.append((ms, cand))
        if log:
            log(f"tune {key}: variant {cand[0]} TY {cand[1]} TZ {cand[2]}: {ms:.4f} ms/step")
    ms, best = min(results)
    value = {"variant": best[0], "tile_y": best[1], "tile_z": best[2], "ms_per_step": ms,
             "candidates": len(cands)}
    store(key, value, path)
    return value


def apply_grid(g: "fdtd.Grid", choice: dict) -> None:
    g.set_kernel(choice["variant"], choice["tile_y"], choice["tile_z"])


def apply_batch(b: "fdtd.Batch", choice: dict, graph_steps: int = 0) -> None:
    b.set_kernel(choice["tile_x"], choice["tile_y"], choice["tile_z"], graph_steps)
    if choice["tile_x"] == 60:
        b.set_persistent(choice.get("persistent", True))


def tune_batch(make_batch, key: str, candidates: Iterable = None, warmup: int = 4, steps: int = 20,
               path: str = None, force: bool = False, log=None) -> dict:
    """make_batch(max_steps) -> an fdtd.Batch, or a Batch with room for
    tuning_steps() more steps.  Returns the best {tile_x, tile_y, tile_z,
    persistent, ms_per_step} (apply it with apply_batch)."""
    cache = load_cache(path)
    if key in cache and not force:
        return cache[key]
    cands = list(candidates or BATCH_CANDIDATES)
    b = make_batch if isinstance(make_batch, fdtd.Batch) else make_batch(len(cands) * (warmup + steps) + 4)
    results = []
    for tx, ty, tz, per in cands:
        b.set_kernel(tx, ty, tz, 0)
        if tx == 60:
            b.set_persistent(bool(per))
        b.run(warmup)
        b.timing(True)
        b.time()
        b.run(steps)
        ms, n = b.time()
        b.timing(False)
        results.append((ms / max(n, 1), (tx, ty, tz, per)))
        if log:
            log(f"tune {key}: tile {tx}x{ty} TZ {tz} persistent {per}: {ms / max(n, 1):.4f} ms/step")
    ms, best = min(results)
    value = {"tile_x": best[0], "tile_y": best[1], "tile_z": best[2], "persistent": bool(best[3]),
             "ms_per_step": ms, "candidates": len(cands)}
    store(key, value, path)
    return value
