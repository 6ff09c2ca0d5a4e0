"""Learned warm start: a network that maps a day's loads to an initial point
of the solver, trained on the solver's own solutions.

    python -m paper_2310_06650_amd.warmstart [--train 256] [--test 16]

The paper starts Adam from a copper-plate dispatch and names machine
learning as future work (Sections III and V).  Here the grid is fixed and the
loads vary from day to day (synth.load_draw); for each training day the plain
solve on the GPU (qg_solve from the flat start) produces a solution, and an
MLP (qg_mlp.h; FP32 training, BF16 inference) learns loads -> solution.  On
held-out days the network's prediction, clipped to the box, starts a shorter
solve, and the time to come within 1 % of the plain solve's best score is
compared with the plain solve's own time to get there.

Everything on the device runs through the library's kernels; this module
marshals arrays, standardises features and targets, and schedules the work.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import sys
import time

import numpy as np

from . import qg, synth

# schedules (qg_solve_opts keywords): the plain solve from the flat start, and
# the solve from a predicted point (penalties at full weight, a narrower
# smoothing range and smaller steps, since it starts near a solution)
PLAIN = dict(alpha0=3e-3, alphaf=1e-5, eps0=1e-1, epsf=1e-4, beta0=0.1, betaf=1.0, rho0=0.1,
             rhof=1.0)
WARM = dict(alpha0=1e-3, alphaf=1e-5, eps0=1e-2, epsf=1e-4, beta0=1.0, betaf=1.0, rho0=1.0,
            rhof=1.0)


def features(case, draw):
    """Input of the network: loads [T*N] then reserve requirements [T]."""
    load_p, _, reserve = draw
    return np.concatenate([np.asarray(load_p).reshape(-1), np.asarray(reserve).reshape(-1)])


def box(case):
    """Lower and upper bounds of x (angles unbounded)."""
    T, N, G = case.n_period, case.n_bus, case.n_gen
    inf = np.inf
    lo = np.concatenate([np.tile(case.v_min, T), np.full(T * N, -inf), np.zeros(T * G),
                         np.tile(case.gen_qmin, T), np.zeros(T * G), np.zeros(T * G)])
    hi = np.concatenate([np.tile(case.v_max, T), np.full(T * N, inf),
                         np.tile(case.gen_pmax, T), np.tile(case.gen_qmax, T),
                         np.tile(case.gen_rmax, T), np.ones(T * G)])
    return lo, hi


class Worker:
    """One problem (arena, workspace, vectors) on its own stream."""

    def __init__(self, case):
        import torch
        self.torch = torch
        self.case = case
        self.stream = torch.cuda.Stream()
        self.prob = qg.Problem(case)
        self.prob.stream = self.stream
        with torch.cuda.stream(self.stream):
            self.x = self.prob.new_vector()
            self.m = self.prob.new_vector()
            self.v = self.prob.new_vector()
        self.stream.synchronize()

    def solve(self, draw, x0, n_steps, sched, z_ed=0.0, stop_ratio=2.0, check_every=0):
        torch = self.torch
        self.prob.update_loads(*draw)
        with torch.cuda.stream(self.stream):
            self.x.copy_(torch.as_tensor(x0))
            self.m.zero_()
            self.v.zero_()
        opts = qg.solve_opts(n_steps, [sched["alpha0"]] * 6, alphaf=[sched["alphaf"]] * 6,
                             n_total=n_steps, eps0=sched["eps0"], epsf=sched["epsf"],
                             beta0=sched["beta0"], betaf=sched["betaf"], rho0=sched["rho0"],
                             rhof=sched["rhof"], z_ed=z_ed, stop_ratio=stop_ratio,
                             check_every=check_every, use_graph=1)
        rep = self.prob.solve(self.x, self.m, self.v, opts)
        self.stream.synchronize()
        return rep

    def close(self):
        self.prob.close()


def flat_for(case, draw):
    return synth.flat_start(synth.with_loads(case, draw))


def generate(case, seeds, n_steps, workers=4):
    """(X, Y): features and plain-solve solutions of the given load draws."""
    pool = [Worker(case) for _ in range(workers)]
    X = np.zeros((len(seeds), case.n_period * (case.n_bus + 1)))
    Y = np.zeros((len(seeds), case.n_x))

    def job(i):
        w = pool[i % workers]
        draw = synth.load_draw(case, seeds[i])
        w.solve(draw, flat_for(case, draw), n_steps, PLAIN)
        X[i] = features(case, draw)
        Y[i] = w.x.cpu().numpy()

    # one thread per worker: jobs of a worker run in order on its stream
    with cf.ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(lambda k=k: [job(i) for i in range(k, len(seeds), workers)])
                for k in range(workers)]
        for f in futs:
            f.result()
    for w in pool:
        w.close()
    return X, Y


class Scaler:
    def __init__(self, A, floor=1e-6):
        self.mu = A.mean(axis=0)
        self.sd = np.maximum(A.std(axis=0), floor)

    def fwd(self, A):
        return (A - self.mu) / self.sd

    def inv(self, A):
        return A * self.sd + self.mu


class WarmStart:
    """Standardisers and the trained network."""

    def __init__(self, case, X, Y, width=512, depth=3, seed=0):
        import torch
        self.torch = torch
        self.case = case
        self.sx, self.sy = Scaler(X), Scaler(Y)
        self.net = qg.MLP(X.shape[1], width, depth, Y.shape[1], max_batch=max(64, len(X)))
        # He-style initialisation drawn on the host and uploaded
        rng = np.random.default_rng(seed)
        flat = np.zeros(self.net.n_params, dtype=np.float32)
        sizes = [X.shape[1]] + [width] * depth + [Y.shape[1]]
        for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
            wo, _ = self.net.offsets(i)
            flat[wo:wo + a * b] = rng.normal(0.0, np.sqrt(2.0 / a), a * b).astype(np.float32)
        self.net.set_params(flat)
        self.Xn = torch.as_tensor(self.sx.fwd(X), dtype=torch.float32).cuda()
        self.Yn = torch.as_tensor(self.sy.fwd(Y), dtype=torch.float32).cuda()

    def train(self, steps, batch=64, lr=1e-3, seed=0):
        rng = np.random.default_rng(seed)
        n = self.Xn.shape[0]
        losses = []
        for it in range(steps):
            idx = self.torch.as_tensor(rng.choice(n, size=min(batch, n), replace=False)).cuda()
            xb = self.Xn.index_select(0, idx).contiguous()
            yb = self.Yn.index_select(0, idx).contiguous()
            loss = self.net.train_step(xb, yb, lr)
            if it % 50 == 0 or it == steps - 1:
                losses.append(float(loss))
        return losses

    def predict(self, draws, bf16=True):
        torch = self.torch
        X = np.stack([features(self.case, d) for d in draws])
        xb = torch.as_tensor(self.sx.fwd(X), dtype=torch.float32).cuda()
        if bf16:
            self.net.to_bf16()
            y = self.net.forward_bf16(xb)
        else:
            y = self.net.forward(xb)
        torch.cuda.synchronize()
        lo, hi = box(self.case)
        return np.clip(self.sy.inv(y.cpu().numpy().astype(np.float64)), lo, hi)


def compare(case, ws, seeds, n_plain=20000, n_warm=4000, check_every=250):
    """Per held-out day: the plain solve's best ratio after n_plain steps, the
    steps and seconds it takes to come within 1 % of it, and the same for
    solves started from the network's prediction (BF16 inference) and, as an
    ablation, from the mean of the training solutions."""
    from . import ed
    w = Worker(case)
    rows = []
    preds = ws.predict([synth.load_draw(case, s) for s in seeds])
    lo, hi = box(case)
    x_mean = np.clip(ws.sy.mu, lo, hi)
    for s, x_pred in zip(seeds, preds):
        draw = synth.load_draw(case, s)
        z_ed = ed.copper_plate(synth.with_loads(case, draw)).z_ed
        best = w.solve(draw, flat_for(case, draw), n_plain, PLAIN).final_score / z_ed
        target = 0.99 * best
        row = dict(seed=int(s), best_ratio=best, target=target)
        for name, x0, n, sched in (("plain", flat_for(case, draw), n_plain, PLAIN),
                                   ("warm", x_pred, n_warm, WARM),
                                   ("mean", x_mean, n_warm, WARM)):
            r = w.solve(draw, x0, n, sched, z_ed=z_ed, stop_ratio=target,
                        check_every=check_every)
            row[name + "_steps"] = int(r.steps_to_gap)
            row[name + "_s"] = r.time_to_gap_s
            row[name + "_final_ratio"] = r.final_score / z_ed
        rows.append(row)
    w.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--solve-steps", type=int, default=8000)
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--depth", type=int, default=3)
    ap.add_argument("--warm-steps", default="4000,8000",
                    help="schedule lengths of the warm solves (comma list)")
    args = ap.parse_args()
    case = synth.config_case(args.config)
    t0 = time.perf_counter()
    X, Y = generate(case, list(range(10000, 10000 + args.train)), args.solve_steps)
    t1 = time.perf_counter()
    print(f"training data: {args.train} days in {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    ws = WarmStart(case, X, Y, width=args.width, depth=args.depth)
    losses = ws.train(args.train_steps)
    t2 = time.perf_counter()
    print(f"trained in {t2 - t1:.1f} s", file=sys.stderr, flush=True)
    runs = {}
    for n_warm in [int(v) for v in args.warm_steps.split(",")]:
        runs[n_warm] = compare(case, ws, list(range(20000, 20000 + args.test)), n_warm=n_warm)
        print(f"compared with {n_warm}-step warm schedules", file=sys.stderr, flush=True)
    t3 = time.perf_counter()
    def med(rows, key):
        v = [r[key] for r in rows if r[key.split("_")[0] + "_steps"] > 0]
        return float(np.median(v)) if v else None

    summary = dict(
        config=args.config, train_days=args.train, test_days=args.test,
        solve_steps=args.solve_steps, net=f"{X.shape[1]}-{args.width}x{args.depth}-{Y.shape[1]}",
        n_params=ws.net.n_params, data_s=t1 - t0, train_s=t2 - t1, eval_s=t3 - t2,
        loss_first=losses[0], loss_last=losses[-1],
        by_warm_schedule={
            n: dict(reached={k: sum(r[k + "_steps"] > 0 for r in rows)
                             for k in ("plain", "warm", "mean")},
                    median_s={k: med(rows, k + "_s") for k in ("plain", "warm", "mean")},
                    median_steps={k: med(rows, k + "_steps") for k in ("plain", "warm", "mean")})
            for n, rows in runs.items()},
        rows={n: rows for n, rows in runs.items()})
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
