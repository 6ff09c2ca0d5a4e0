"""Many independent scenarios of uneven size on one GPU.

    python -m paper_2310_06650_amd.batch [--n 64] [--steps 200]

Builds the scenarios of synth.batch_cases (bus counts 100..2000, 12..48
periods, every non-islanding outage), picks each one's contingency tile with
the autotuner, and measures the same number of Adam steps two ways: each
scenario solved alone in turn (its own step graphs), and all of them in one
batched solve (qg_solve_batch: six launches per step for the whole batch,
the contingency map-reduce persistent over a work list, 16 steps per graph).
Prints one JSON line with scenario-steps per second, contingency elements per
second and the effective rate of outage-factor bytes.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import autotune, qg, synth


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tile", default="s4x4",
                    help="tile of every scenario with --no-tune (4 wavefronts of 4 periods)")
    args = ap.parse_args()
    import torch
    cases = synth.batch_cases(args.n, seed0=args.seed)
    t0 = time.perf_counter()
    probs = [qg.Problem(c) for c in cases]
    build_s = time.perf_counter() - t0
    x0s = [synth.flat_start(c) for c in cases]
    tiles = []
    t0 = time.perf_counter()
    for p, x0, c in zip(probs, x0s, cases):
        if args.no_tune:
            if p.K > 0:
                p.set_tile(args.tile)
            tiles.append(p.tile())
            continue
        tile, _ = autotune.tune(p, p.new_vector(x0), steps=32, batch=True)
        tiles.append(tile)
    tune_s = time.perf_counter() - t0
    opts = qg.solve_opts(args.steps, [3e-3] * 6, alphaf=[1e-5] * 6, n_total=args.steps,
                         eps0=1e-1, epsf=1e-4, beta0=0.1, betaf=1.0, rho0=0.1, rhof=1.0,
                         use_graph=1)
    xs = [p.new_vector(x0) for p, x0 in zip(probs, x0s)]
    ms = [p.new_vector() for p in probs]
    vs = [p.new_vector() for p in probs]

    def reset():
        for x, m, v, x0 in zip(xs, ms, vs, x0s):
            x.copy_(torch.from_numpy(x0).to(x.device))
            m.zero_()
            v.zero_()
        torch.cuda.synchronize()

    # one after another (graphs captured in a first pass)
    for p, x, m, v in zip(probs, xs, ms, vs):
        p.solve(x, m, v, opts)
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, x, m, v in zip(probs, xs, ms, vs):
        p.solve(x, m, v, opts)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    x_seq = [x.cpu().numpy().copy() for x in xs]
    # batched
    reset()
    reps = qg.solve_batch(probs, xs, ms, vs, opts)
    torch.cuda.synchronize()
    batch_s = reps[0].wall_s
    same = all(np.array_equal(a, x.cpu().numpy()) for a, x in zip(x_seq, xs))
    elems = sum(c.n_period * c.n_branch * c.n_ctg for c in cases)
    lodf_bytes = sum(p.dims["Lp"] * p.dims["Kp"] * 8 for p in probs)
    out = dict(
        scenarios=args.n, steps=args.steps,
        buses=int(sum(c.n_bus for c in cases)), periods_mean=float(np.mean([c.n_period for c in cases])),
        contingency_elements_per_step=int(elems), lodf_bytes=int(lodf_bytes),
        build_s=build_s, tune_s=tune_s,
        tiles={f"{c.n_bus}x{c.n_period}": t for c, t in zip(cases, tiles)},
        sequential=dict(seconds=seq_s, scenario_steps_per_s=args.n * args.steps / seq_s,
                        elements_per_s=elems * args.steps / seq_s),
        batched=dict(seconds=batch_s, scenario_steps_per_s=args.n * args.steps / batch_s,
                     elements_per_s=elems * args.steps / batch_s,
                     lodf_once_per_step_GBps=lodf_bytes * args.steps / batch_s / 1e9),
        batched_equals_sequential=bool(same))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
