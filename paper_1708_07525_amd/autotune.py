"""Launch-shape autotuning with a persistent cache.

``lbm_autotune`` (C ABI) times every supported tile shape, cache policy and steps-per-launch
count of the step kernels
on a context, keeps the fastest and restores the state it started from.  This module keys the
winner by GPU, storage precision, lattice size class, porosity kind and wall family, stores it in a JSON
file, and applies the cached choice to later contexts of the same class without re-timing.
Results never depend on the tile shape or the cache policy (the per-node arithmetic is one
function), only the speed does.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbm_dd", "autotune.json")
# part of every key: raised when the kernels' launch choices change (three steps per launch for
# FP32, a three-step tile with its rest populations in registers, the tile order of the
# multi-step launches, their taller tiles), so that choices timed with older kernels are not
# applied to newer ones
KERNEL_GENERATION = 4


def cache_path() -> str:
    return os.environ.get("LBM_AUTOTUNE_CACHE", DEFAULT_CACHE)


def size_class(n: int) -> int:
    """Smallest power of two >= n (lattices of one class share a tuned shape)."""
    c = 1
    while c < n:
        c *= 2
    return c


def key(device_name: str, precision: str, nx: int, ny: int, porosity_field: bool, node_walls: bool = False) -> str:
    k = (f"g{KERNEL_GENERATION}|{device_name}|{precision}|{size_class(nx)}x{size_class(ny)}|"
         f"{'field' if porosity_field else 'uniform'}")
    return k + "|node-walls" if node_walls else k


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(solver, device_name: str, porosity_field: bool, steps: int = 20, path: str | None = None,
         force: bool = False, node_walls: bool = False):
    """Apply the cached tile shape, cache policy, steps per launch, strip width and multi-step
    tile rows for this solver's class (walls through the boundary nodes are a class of their own), or
    time all of them and cache the fastest.  Returns (tile_x, tile_y), ms_per_step (None when taken from the cache)."""
    k = key(device_name, solver.precision, solver.nx, solver.ny, porosity_field, node_walls)
    entries = load(path)
    if not force and k in entries:
        tx, ty = entries[k]["tile"]
        solver.set_tile(tx, ty)
        solver.set_cache_policy(int(entries[k].get("policy", -1)))
        solver.set_steps_per_launch(int(entries[k].get("steps_per_launch", 0)))
        solver.set_strip_width(int(entries[k].get("strip_width", -1)))
        solver.set_tile_rows(int(entries[k].get("tile_rows", 0)))
        return (tx, ty), None
    (tx, ty), ms = solver.autotune(steps)
    entries = load(path)          # re-read: another process may have added entries
    entries[k] = {"tile": [tx, ty], "policy": solver.get_cache_policy(),
                  "steps_per_launch": solver.get_steps_per_launch(), "strip_width": solver.get_strip_width(),
                  "tile_rows": solver.get_tile_rows(),
                  "ms_per_step": ms, "steps": steps}
    store(entries, path)
    return (tx, ty), ms
