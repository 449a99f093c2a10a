"""Autotuner for the batched propagator's per-group tiling.

For every group it times a few RK4 steps of that group alone for each
(tile, rows_per_item) candidate and keeps the fastest.  Results are cached in
a JSON file keyed by device name, N, number of instances and number of terms
(path from $SUN_AUTOTUNE_CACHE, default ~/.cache/sunbloch/autotune.json).
The tiling never changes the numbers, only the speed.
"""

from __future__ import annotations

import json
import os
import time

import torch

TILES = (16, 32, 64)
ROWS = (32, 64, 128)


def cache_path() -> str:
    return os.environ.get("SUN_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sunbloch", "autotune.json"))


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _key(G) -> str:
    name = torch.cuda.get_device_name(0).replace(" ", "_")
    return f"{name}|N={G['N']}|B={G['B']}|nt={G['nt']}|lds"


def autotune_batched(bp, tiles=TILES, rows=ROWS, probe_steps: int = 6, use_cache: bool = True,
                     log=None) -> dict:
    """Pick (tile, rows_per_item) per group of a BatchedPropagator.  The
    group states are saved and restored (step counters reset to 0)."""
    path = cache_path()
    cache = _load(path) if use_cache else {}
    chosen = {}
    for g, G in enumerate(bp.groups):
        key = _key(G)
        if use_cache and key in cache:
            t, r = cache[key]["tile"], cache[key]["rows_per_item"]
            bp.tune(g, t, r)
            chosen[g] = {"tile": t, "rows_per_item": r, "cached": True}
            continue
        saved = bp.get_state(g)
        best = None
        steps = min(probe_steps, max(1, G["steps"]))
        for t in tiles:
            for r in rows:
                bp.tune(g, t, r)
                bp.set_state(g, saved)
                bp.run(1, only_group=g)            # warm
                t0 = time.perf_counter()
                bp.run(steps, only_group=g)
                el = time.perf_counter() - t0
                if best is None or el < best[0]:
                    best = (el, t, r)
        _, t, r = best
        bp.tune(g, t, r)
        bp.set_state(g, saved)
        chosen[g] = {"tile": t, "rows_per_item": r, "cached": False, "probe_s_per_step": best[0] / steps}
        cache[key] = {"tile": t, "rows_per_item": r}
        if log:
            log(f"autotune group {g} (N={G['N']}, B={G['B']}): tile={t} rows={r}")
    if use_cache:
        _save(path, cache)
    return chosen
