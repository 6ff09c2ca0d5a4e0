"""Contingency screening (Alg. 2) against the exact path: speed and accuracy.

    python -m paper_2310_06650_amd.screening [--config c2] [--steps 20000]

Solves the same schedule from the flat start with every contingency scored
(the exact path) and with screening at several settings (worst fraction,
random fraction, steps between exact refresh steps).  For each run: steps per
second over the whole solve (refresh steps and set selections included), the
final score (always evaluated with every contingency) relative to the
copper-plate bound z_ed, and the time to come within 1 % of the exact
solve's best ratio.  Also the per-kernel times of one exact and one screened
step of the contingency stages at the final point, and how many contingencies
overload anything there.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import ed, qg, synth

SETTINGS = [(0.02, 0.02, 25), (0.05, 0.05, 25), (0.1, 0.05, 25), (0.1, 0.1, 10),
            (0.2, 0.1, 50)]
SCHEDULE = dict(eps0=1e-1, epsf=1e-4, beta0=0.1, betaf=1.0, rho0=0.1, rhof=1.0)
ALPHA0, ALPHAF = [3e-3] * 6, [1e-5] * 6


def solve(prob, case, n_steps, z_ed, stop_ratio=2.0, check_every=0):
    import torch
    x = prob.new_vector(synth.flat_start(case))
    m, v = prob.new_vector(), prob.new_vector()
    torch.cuda.synchronize()
    rep = prob.solve(x, m, v, qg.solve_opts(n_steps, ALPHA0, ALPHAF, n_total=n_steps, z_ed=z_ed,
                                            stop_ratio=stop_ratio, check_every=check_every,
                                            use_graph=1, **SCHEDULE))
    return rep, x


def stage_us(prob, x, reps=50):
    return {qg.KERNEL_NAMES[s]: prob.time_stage(x, s, reps, 1e-4) for s in (1, 2, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args()
    case = synth.config_case(args.config)
    z_ed = ed.copper_plate(case).z_ed
    prob = qg.Problem(case)
    K = prob.K
    out = dict(config=args.config, workload=f"{case.n_bus}-bus x {case.n_period}-period x "
                                            f"{K}-contingency synthetic grid",
               steps=args.steps, z_ed=z_ed, runs=[])

    solve(prob, case, 64, z_ed)                      # graph capture and warm-up
    rep, x = solve(prob, case, args.steps, z_ed)
    best = rep.final_score / z_ed
    target = 0.99 * best
    gap, _ = solve(prob, case, args.steps, z_ed, stop_ratio=target, check_every=250)
    exact_us = stage_us(prob, x)
    prob.set_screening(top_frac=1.0)
    prob.screen_refresh(x, 1e-4, 1.0, 1.0)
    _, sev = prob.active_contingencies(severities=True)
    prob.set_screening(None)
    out["exact"] = dict(steps_per_s=args.steps / rep.wall_s, final_ratio=best,
                        target_ratio=target, steps_to_target=int(gap.steps_to_gap),
                        time_to_target_s=gap.time_to_gap_s, stage_us=exact_us,
                        overloading_at_end=int((sev > 0).sum()))
    print(f"exact: {out['exact']['steps_per_s']:.0f} steps/s", file=sys.stderr, flush=True)
    for top, rand, refresh in SETTINGS:
        prob.set_screening(top_frac=top, rand_frac=rand, zeta=0.0, refresh=refresh,
                           seed=args.seed)
        solve(prob, case, 64, z_ed)
        rep, x = solve(prob, case, args.steps, z_ed)
        gap, _ = solve(prob, case, args.steps, z_ed, stop_ratio=target, check_every=250)
        n_act = len(prob.active_contingencies())
        out["runs"].append(dict(
            top_frac=top, rand_frac=rand, refresh=refresh, n_act=n_act,
            steps_per_s=args.steps / rep.wall_s,
            speedup=(args.steps / rep.wall_s) / out["exact"]["steps_per_s"],
            final_ratio=rep.final_score / z_ed,
            final_vs_exact=(rep.final_score / z_ed) / best,
            steps_to_target=int(gap.steps_to_gap), time_to_target_s=gap.time_to_gap_s,
            screened_stage_us=stage_us(prob, x)))
        print(f"screening {top}/{rand}/{refresh}: {out['runs'][-1]['speedup']:.2f}x, final "
              f"{out['runs'][-1]['final_vs_exact']:.4f} of exact", file=sys.stderr, flush=True)
        prob.set_screening(None)
    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
