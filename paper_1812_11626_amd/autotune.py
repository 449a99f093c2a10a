"""Autotuner for the batched propagator's per-group tiling.

For every group it times a few RK4 steps of that group alone for each
(tile, rows_per_item) candidate and keeps the fastest; then it times the
whole batch with those choices against a few uniform tilings and keeps the
fastest of these.  Results are cached in
a JSON file keyed by device name, N, number of instances and number of terms
(path from $SUN_AUTOTUNE_CACHE, default ~/.cache/sunbloch/autotune.json).
The tiling never changes the numbers, only the speed.
"""

from __future__ import annotations

import json
import os
import time

import torch

TILES = (16, 32, 64, 128)
ROWS = (32, 64, 128)
UNIFORM = ((128, 64), (128, 32), (64, 64))


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
    return f"{name}|N={G['N']}|B={G['B']}|nt={G['nt']}|lds2"


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
    # Whole-batch check: the per-group choices against a few uniform tilings,
    # timed on all groups together (one launch per stage covers every group,
    # and mixing 128-instance tiles with narrower ones costs a second launch).
    bkey = "batch|" + ";".join(_key(G) for G in bp.groups)
    if use_cache and bkey in cache:
        pick = cache[bkey]
    else:
        saved = [bp.get_state(g) for g in range(len(bp.groups))]
        steps = min(probe_steps, max(1, min(G["steps"] for G in bp.groups)))
        cands = [[(chosen[g]["tile"], chosen[g]["rows_per_item"]) for g in range(len(bp.groups))]]
        cands += [[(t, r)] * len(bp.groups) for (t, r) in UNIFORM if t in tiles]
        best = None
        for cand in cands:
            for g, (t, r) in enumerate(cand):
                bp.tune(g, t, r)
                bp.set_state(g, saved[g])
            bp.run(1)                                  # warm
            t0 = time.perf_counter()
            bp.run(steps)
            el = time.perf_counter() - t0
            if best is None or el < best[0]:
                best = (el, cand)
        pick = [list(x) for x in best[1]]
        for g in range(len(bp.groups)):
            bp.set_state(g, saved[g])
        cache[bkey] = pick
    for g, (t, r) in enumerate(pick):
        bp.tune(g, t, r)
        if (t, r) != (chosen[g]["tile"], chosen[g]["rows_per_item"]):
            chosen[g] = {"tile": t, "rows_per_item": r, "cached": chosen[g]["cached"], "whole_batch": True}
            if log:
                log(f"autotune group {g}: whole-batch choice tile={t} rows={r}")
    if use_cache:
        _save(path, cache)
    return chosen
