"""Tile autotuner of the contingency map-reduce.

The tile (period-split: wavefronts per block, periods per wavefront, branch
tiles per block; branch-stacked: branches per wavefront, wavefronts per
block, periods per block, branch tiles per block) trades the re-reads of the
outage factors, the partial sums and the per-block fixed costs against the
number of blocks in flight; the best choice depends on the grid's shape.
Tiles are named by their text form (``Problem.tile``).  ``tune`` times, for
each candidate, a short graph-replayed solve from a copy of the given point
(the whole step: the tile also changes how much the reductions after the
map-reduce read, and the kernels' overlap) -- or, with measure="stages", the
three kernels the tile affects with qg_time_stage -- and keeps the fastest;
results are cached per shape class (padded branch and contingency counts,
periods, factor storage) in a JSON file ($QG_AUTOTUNE_CACHE, default
~/.cache/qg/autotune.json).
"""
from __future__ import annotations

import json
import os

from . import qg

# text forms; a missing lt: the library's default for the rest of the tile
CANDIDATES = ["s4x2", "s4x4", "s2x2", "s3x2", "s8x2", "s4x3", "s4x6", "s8x6", "s4x4x16",
              "s4x2x4", "s1x4", "s1x4x8", "s1x4x12", "s2x4x8", "s3x4x8", "s4x2x16",
              "8x8x4", "8x4x4", "8x8x7", "16x4x4", "8x8x4x1", "8x8x7x4", "8x4x8x8"]
# the tiles a batched solve takes (4 wavefronts of 4 periods; branch tiles
# per block free).  In a batch the map-reduce's blocks are work items of a
# persistent launch, each with a fixed cost at its start, so the candidates
# are the larger items, timed through the batched path.
BATCH_CANDIDATES = ["s4x4x8", "s4x4x16", "s4x4x32"]


def cache_path():
    return os.environ.get("QG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "qg", "autotune.json"))


def shape_key(prob, batch=False):
    d = prob.dims
    return f"Lp{d['Lp']}-Kp{d['Kp']}-T{d['T']}-lodf{d['lodf_kind']}" + ("-batch" if batch else "")


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


def step_us(prob, x, steps=64, eps=1e-2, batch=False):
    """Microseconds per step of a graph-replayed solve of ``steps`` steps from
    a copy of x (small fixed step sizes and homotopy), after one untimed solve
    that captures the graph; batch=True: through the batched path (the
    problem alone in a batch).  x itself is not changed."""
    xs = x.clone()
    m, v = prob.new_vector(), prob.new_vector()
    opts = qg.solve_opts(steps, [1e-5] * qg.QG_NCLASS, n_total=steps, eps0=eps, epsf=eps,
                         use_graph=1)
    run = ((lambda: qg.solve_batch([prob], [xs], [m], [v], opts)[0]) if batch
           else (lambda: prob.solve(xs, m, v, opts)))
    run()
    xs.copy_(x)
    m.zero_()
    v.zero_()
    rep = run()
    return rep.wall_s / steps * 1e6


def tune(prob, x, reps=30, eps=1e-2, candidates=None, use_cache=True, measure="step",
         steps=64, batch=False):
    """Set the fastest tile on prob (timed at the point x) and return
    (tile, {tile: microseconds}): per step of a short solve (measure="step")
    or the sum of the three contingency kernels (measure="stages", reps
    launches each).  batch=True: among the tiles a batched solve takes."""
    key = shape_key(prob, batch)
    if candidates is None and batch:
        candidates = BATCH_CANDIDATES
    cache = _load() if use_cache else {}
    hit = cache.get(key)
    if use_cache and hit and isinstance(hit.get("tile"), str) and hit.get("measure") == measure:
        prob.set_tile(hit["tile"])
        return hit["tile"], hit["times"]
    times = {}
    for cand in (candidates or CANDIDATES):
        try:
            prob.set_tile(cand)
        except qg.QgError:
            continue
        if measure == "step":
            us = step_us(prob, x, steps, eps, batch=batch)
        else:
            us = sum(prob.time_stage(x, s, reps, eps) for s in (1, 2, 3))
        times[prob.tile()] = us
    tile = min(times, key=times.get)
    prob.set_tile(tile)
    if use_cache:
        cache[key] = dict(tile=tile, times=times, measure=measure)
        _save(cache)
    return tile, times
