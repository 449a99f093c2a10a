"""Autotuner for the batched propagator's per-group tiling.

For every group it times a few RK4 steps of that group alone for each
(tile, rows_per_item, path) candidate and keeps the fastest; then it times
the whole batch with those choices against a few uniform tilings and keeps
the fastest of these.  Results are cached in
a JSON file keyed by device architecture and compute-unit count, N, number
of instances and number of terms
(path from $SUN_AUTOTUNE_CACHE, default ~/.cache/sunbloch/autotune.json).
The tiling never changes the numbers, only the speed.
"""

from __future__ import annotations

import json
import os
import time

import torch

from ._lib import SunError

TILES = (16, 32, 64, 128)
ROWS = (32, 64, 128)
# path 0: LDS-staged row blocks, one instance per lane below 128-instance
# tiles; path 2: the same with two instances per lane for every tile width;
# path 3: path 2 with the gathered state rows staged in LDS (tiles 8-32)
# path 4: instance-major state on a segmented sliced layout, 4 or 8 instances
# per wavefront (the tile value); rows_per_item does not apply
# path 5: one wavefront per (row, tile of 64 or 128 instances), the matrix
# read through the scalar cache, rows swept in order per XCD; rows_per_item
# does not apply
# path 7: persistent workgroups with pipelined LDS staging of each block's
# state rows, tiles of 64; rows_per_item is the block's row limit (<= 32)
PATHS = (0, 2, 3, 4, 5, 7)
TILES3 = (8, 16, 32)
TILES4 = (4, 8)
TILES5 = (64, 128)
ROWS7 = (16, 32)
UNIFORM = ((128, 64, 0), (128, 32, 0), (64, 64, 0), (16, 64, 2), (32, 64, 2), (16, 128, 3), (8, 128, 3),
           (4, 64, 4), (8, 64, 4), (128, 64, 5), (64, 64, 5), (64, 32, 7))


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


def _device_tag() -> str:
    """Architecture and compute-unit count of device 0 (the marketing name is
    not used: some profilers report it empty)."""
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "") or "unknown"
    return f"{arch.split(':')[0]}-{props.multi_processor_count}cu"


def _key(G) -> str:
    return f"{_device_tag()}|N={G['N']}|B={G['B']}|nt={G['nt']}|lds4|p7"


def _candidates(tiles, rows, paths):
    out = []
    for p in paths:
        if p == 4:
            out += [(t, 64, 4) for t in TILES4]
            continue
        if p == 5:
            out += [(t, 64, 5) for t in TILES5]
            continue
        if p == 7:
            out += [(64, r, 7) for r in ROWS7]
            continue
        for t in (TILES3 if p == 3 else tiles):
            if p == 2 and t == 128:
                continue               # 128-instance tiles are two per lane on path 0 already
            for r in rows:
                out.append((t, r, p))
    return out


def autotune_batched(bp, tiles=TILES, rows=ROWS, paths=PATHS, probe_steps: int = 6, use_cache: bool = True,
                     log=None) -> dict:
    """Pick (tile, rows_per_item, path) per group of a BatchedPropagator.
    The group states are saved and restored (step counters reset to 0)."""
    path = cache_path()
    cache = _load(path) if use_cache else {}
    chosen = {}
    for g, G in enumerate(bp.groups):
        key = _key(G)
        if use_cache and key in cache:
            t, r, p = cache[key]["tile"], cache[key]["rows_per_item"], cache[key]["path"]
            bp.tune(g, t, r, p)
            chosen[g] = {"tile": t, "rows_per_item": r, "path": p, "cached": True}
            continue
        saved = bp.get_state(g)
        best = None
        steps = min(probe_steps, max(1, G["steps"]))
        for (t, r, p) in _candidates(tiles, rows, paths):
            try:
                bp.tune(g, t, r, p)
            except SunError:
                continue                        # path 4 needs 1-3 instance-dependent terms
            bp.set_state(g, saved)
            bp.run(1, only_group=g)            # warm
            t0 = time.perf_counter()
            bp.run(steps, only_group=g)
            el = time.perf_counter() - t0
            if best is None or el < best[0]:
                best = (el, t, r, p)
        _, t, r, p = best
        bp.tune(g, t, r, p)
        bp.set_state(g, saved)
        chosen[g] = {"tile": t, "rows_per_item": r, "path": p, "cached": False, "probe_s_per_step": best[0] / steps}
        cache[key] = {"tile": t, "rows_per_item": r, "path": p}
        if log:
            log(f"autotune group {g} (N={G['N']}, B={G['B']}): tile={t} rows={r} path={p}")
    # Whole-batch check: the per-group choices against a few uniform tilings,
    # timed on all groups together (one launch per stage covers every group,
    # and mixing 128-instance tiles with narrower ones costs a second launch).
    bkey = "batch|" + ";".join(_key(G) for G in bp.groups)
    if use_cache and bkey in cache:
        pick = cache[bkey]
    else:
        saved = [bp.get_state(g) for g in range(len(bp.groups))]
        steps = min(probe_steps, max(1, min(G["steps"] for G in bp.groups)))
        cands = [[(chosen[g]["tile"], chosen[g]["rows_per_item"], chosen[g]["path"]) for g in range(len(bp.groups))]]
        cands += [[(t, r, p)] * len(bp.groups) for (t, r, p) in UNIFORM
                  if (t in TILES3 if p == 3 else (t in TILES4 if p == 4 else
                      (t in TILES5 if p == 5 else (t == 64 if p == 7 else t in tiles))))
                  and p in paths]
        best = None
        for cand in cands:
            try:
                for g, (t, r, p) in enumerate(cand):
                    bp.tune(g, t, r, p)
                    bp.set_state(g, saved[g])
            except SunError:
                continue
            for g in range(len(bp.groups)):
                bp.set_state(g, saved[g])
            bp.run(1)                                  # warm
            el = None
            for _ in range(2):                         # the better of two timings
                t0 = time.perf_counter()
                bp.run(steps)
                t = time.perf_counter() - t0
                el = t if el is None else min(el, t)
                for g in range(len(bp.groups)):
                    bp.set_state(g, saved[g])
            if best is None or el < best[0]:
                best = (el, cand)
        pick = [list(x) for x in best[1]]
        for g in range(len(bp.groups)):
            bp.set_state(g, saved[g])
        cache[bkey] = pick
    for g, (t, r, p) in enumerate(pick):
        bp.tune(g, t, r, p)
        if (t, r, p) != (chosen[g]["tile"], chosen[g]["rows_per_item"], chosen[g]["path"]):
            chosen[g] = {"tile": t, "rows_per_item": r, "path": p, "cached": chosen[g]["cached"], "whole_batch": True}
            if log:
                log(f"autotune group {g}: whole-batch choice tile={t} rows={r} path={p}")
    if use_cache:
        _save(path, cache)
    return chosen
