"""Tile autotuner of the contingency map-reduce.

The tile (branches per wavefront, wavefronts per block, periods per block,
branch tiles per block) trades the re-reads of the outage factors and the
per-block fixed costs against the number of blocks in flight; the best
choice depends on the grid's shape.  ``tune`` times the
three kernels the tile affects (map-reduce, per-contingency and per-branch
reductions) for each candidate with qg_time_stage at a given point and keeps
the fastest; results are cached per shape class (padded branch and
contingency counts, periods, factor storage) in a JSON file
($QG_AUTOTUNE_CACHE, default ~/.cache/qg/autotune.json).
"""
from __future__ import annotations

import json
import os

from . import qg

# (bl, wl, tc, lt); lt 0: the library's default for the other three
CANDIDATES = [(8, 8, 2, 0), (8, 4, 2, 0), (8, 8, 4, 0), (8, 4, 4, 0), (8, 8, 7, 0), (8, 4, 8, 0),
              (16, 4, 2, 0), (16, 4, 4, 0), (8, 2, 4, 0), (16, 2, 8, 0), (8, 8, 4, 1),
              (8, 8, 7, 4), (8, 4, 8, 4), (8, 4, 8, 8)]


def cache_path():
    return os.environ.get("QG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "qg", "autotune.json"))


def shape_key(prob):
    d = prob.dims
    return f"Lp{d['Lp']}-Kp{d['Kp']}-T{d['T']}-lodf{d['lodf_kind']}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(prob, x, reps=30, eps=1e-2, candidates=None, use_cache=True):
    """Set the fastest tile on prob (timed at the point x) and return
    (tile, {tile: microseconds})."""
    key = shape_key(prob)
    cache = _load() if use_cache else {}
    if use_cache and key in cache and len(cache[key]["tile"]) == 4:
        tile = tuple(cache[key]["tile"])
        prob.set_ctg_tile(*tile[:3], lt=tile[3])
        return tile, cache[key]["times"]
    times = {}
    for bl, wl, tc, lt in (candidates or CANDIDATES):
        try:
            prob.set_ctg_tile(bl, wl, tc, lt=lt)
        except qg.QgError:
            continue
        us = sum(prob.time_stage(x, s, reps, eps) for s in (1, 2, 3))
        d = prob.dims
        times[f"{bl}x{wl}x{d['ctg_tc']}x{d['ctg_lt']}"] = us
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split("x"))
    prob.set_ctg_tile(*tile[:3], lt=tile[3])
    if use_cache:
        cache[key] = dict(tile=list(tile), times=times)
        _save(cache)
    return tile, times
