"""Learned warm start: a network that maps a day's loads to an initial point
of the solver, trained on the solver's own solutions.

    python -m paper_2310_06650_amd.warmstart [--train 2000] [--test 200]

The paper starts Adam from the copper-plate dispatch (Section III) and names
machine learning as future work (Section V).  Here the grid is fixed and the
loads vary from day to day (synth.load_draw).  For each training day the
plain solve produces a solution (same-grid days solved together through the
batched step, qg_solve_batch); an MLP (qg_mlp.h; FP32 training, BF16
inference) learns loads -> solution.

On held-out days the network's prediction, clipped to the box, starts the
solver, and is compared with three other starts under the same schedules and
horizons, so that the network's own gain is measured apart from the
schedule's: the flat start (v = 1, theta = 0, u = 1, proportional p), the
copper-plate start (the LP dispatch p, q, r, u of the relaxation with
v = 1, theta = 0) and the mean of the training solutions.  The yardstick of
every run is the same: 0.99 x the score of the plain solve (flat start, plain
schedule) after its full horizon, as a ratio to the copper-plate bound z_ed;
a run stops at the first checked step that reaches it.

Everything on the device runs through the library's kernels; this module
marshals arrays, standardises features and targets, shuffles the training
set on the host, and schedules the work.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import sys
import time

import numpy as np

from . import qg, synth

# schedules (qg_solve_opts keywords): the plain solve's (long, starting with
# soft penalties and wide smoothing) and a short one for starts near a
# solution (penalties at full weight, narrower smoothing, smaller steps)
PLAIN = dict(alpha0=3e-3, alphaf=1e-5, eps0=1e-1, epsf=1e-4, beta0=0.1, betaf=1.0, rho0=0.1,
             rhof=1.0)
WARM = dict(alpha0=1e-3, alphaf=1e-5, eps0=1e-2, epsf=1e-4, beta0=1.0, betaf=1.0, rho0=1.0,
            rhof=1.0)
STARTS = ("flat", "copper", "mean", "net")


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


def opts_for(sched, n_steps, z_ed=0.0, stop_ratio=2.0, check_every=0, skip_final=0):
    return qg.solve_opts(n_steps, [sched["alpha0"]] * 6, alphaf=[sched["alphaf"]] * 6,
                         n_total=n_steps, eps0=sched["eps0"], epsf=sched["epsf"],
                         beta0=sched["beta0"], betaf=sched["betaf"], rho0=sched["rho0"],
                         rhof=sched["rhof"], z_ed=z_ed, stop_ratio=stop_ratio,
                         check_every=check_every, use_graph=1, skip_final=skip_final)


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
        rep = self.prob.solve(self.x, self.m, self.v,
                              opts_for(sched, n_steps, z_ed, stop_ratio, check_every))
        self.stream.synchronize()
        return rep

    def close(self):
        self.prob.close()


def flat_for(case, draw):
    return synth.flat_start(synth.with_loads(case, draw))


def copper_for(case, lp):
    """The copper-plate start: the LP's p, q, r, u; v = 1 and theta = 0."""
    T, N = case.n_period, case.n_bus
    return np.concatenate([np.ones(T * N), np.zeros(T * N),
                           np.asarray(lp.p).reshape(-1), np.asarray(lp.q).reshape(-1),
                           np.asarray(lp.r).reshape(-1), np.asarray(lp.u).reshape(-1)])


def generate(case, seeds, n_steps, batch=64, tile="s4x4x8", log=None):
    """(X, Y): features and plain-solve solutions of the given load draws,
    solved batch days at a time through the batched step (each problem of the
    batch is the same grid with that day's loads)."""
    import torch
    nb = min(batch, len(seeds))
    probs = [qg.Problem(case) for _ in range(nb)]
    for p in probs:
        if p.K > 0:
            p.set_tile(tile)
    xs = [p.new_vector() for p in probs]
    ms = [p.new_vector() for p in probs]
    vs = [p.new_vector() for p in probs]
    X = np.zeros((len(seeds), case.n_period * (case.n_bus + 1)))
    Y = np.zeros((len(seeds), case.n_x))
    opts = opts_for(PLAIN, n_steps)
    for b0 in range(0, len(seeds), nb):
        idx = list(range(b0, min(b0 + nb, len(seeds))))
        for p, x, m, v, i in zip(probs, xs, ms, vs, idx):
            draw = synth.load_draw(case, seeds[i])
            p.update_loads(*draw)
            x.copy_(torch.as_tensor(flat_for(case, draw)))
            m.zero_()
            v.zero_()
            X[i] = features(case, draw)
        torch.cuda.synchronize()
        k = len(idx)
        qg.solve_batch(probs[:k], xs[:k], ms[:k], vs[:k], opts)
        torch.cuda.synchronize()
        for x, i in zip(xs, idx):
            Y[i] = x.cpu().numpy()
        if log:
            log(f"training data: {idx[-1] + 1} of {len(seeds)} days")
    for p in probs:
        p.close()
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

    def __init__(self, case, X, Y, width=512, depth=3, seed=0, batch=64):
        import torch
        self.torch = torch
        self.case = case
        self.batch = batch
        self.sx, self.sy = Scaler(X), Scaler(Y)
        self.net = qg.MLP(X.shape[1], width, depth, Y.shape[1], max_batch=max(batch, 64))
        # He-style initialisation drawn on the host and uploaded
        rng = np.random.default_rng(seed)
        flat = np.zeros(self.net.n_params, dtype=np.float32)
        sizes = [X.shape[1]] + [width] * depth + [Y.shape[1]]
        for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
            wo, _ = self.net.offsets(i)
            flat[wo:wo + a * b] = rng.normal(0.0, np.sqrt(2.0 / a), a * b).astype(np.float32)
        self.net.set_params(flat)
        self.Xn = self.sx.fwd(X).astype(np.float32)
        self.Yn = self.sy.fwd(Y).astype(np.float32)

    def train(self, steps, lr=1e-3, seed=0):
        """Adam on mini-batches of a per-epoch host shuffle: each epoch's
        permuted copy of the standardised set is uploaded once and the
        batches are contiguous slices of it."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        n = self.Xn.shape[0]
        bs = min(self.batch, n)
        # batches start at multiples of 64 rows of FP32, so on 256-byte
        # boundaries as the network's entry points require
        assert bs % 64 == 0 or bs == n, "batch must be a multiple of 64 rows"
        per_epoch = n // bs
        losses = []
        it = 0
        while it < steps:
            perm = rng.permutation(n)
            xe = torch.as_tensor(self.Xn[perm]).cuda()
            ye = torch.as_tensor(self.Yn[perm]).cuda()
            for q in range(per_epoch):
                if it >= steps:
                    break
                loss = self.net.train_step(xe[q * bs:(q + 1) * bs], ye[q * bs:(q + 1) * bs], lr)
                if it % 50 == 0 or it == steps - 1:
                    losses.append(float(loss))
                it += 1
        return losses

    def predict(self, draws, bf16=True):
        torch = self.torch
        X = np.stack([features(self.case, d) for d in draws])
        out = []
        for b0 in range(0, len(X), self.batch):
            xb = torch.as_tensor(self.sx.fwd(X[b0:b0 + self.batch]), dtype=torch.float32).cuda()
            if bf16:
                self.net.to_bf16()
                y = self.net.forward_bf16(xb)
            else:
                y = self.net.forward(xb)
            torch.cuda.synchronize()
            out.append(y.cpu().numpy().astype(np.float64))
        lo, hi = box(self.case)
        return np.clip(self.sy.inv(np.concatenate(out)), lo, hi)


def compare(case, ws, seeds, n_plain=20000, n_warm=4000, check_every=250, workers=4,
            log=None):
    """Per held-out day: z_ed and the copper-plate dispatch (host LP), the
    plain solve's score after n_plain steps (its best), then, for every start
    (flat, copper-plate, mean of the training solutions, network) and both
    schedules (plain: n_plain steps; warm: n_warm steps), the steps and
    seconds to come within 1 % of that best (-1: not reached)."""
    from . import ed
    preds = ws.predict([synth.load_draw(case, s) for s in seeds])
    lo, hi = box(case)
    x_mean = np.clip(ws.sy.mu, lo, hi)
    pool = [Worker(case) for _ in range(workers)]
    rows = [None] * len(seeds)
    done = [0]

    def job(k, w):
        s = seeds[k]
        draw = synth.load_draw(case, s)
        t0 = time.perf_counter()
        lp = ed.copper_plate(synth.with_loads(case, draw))
        lp_s = time.perf_counter() - t0
        z_ed = lp.z_ed
        starts = dict(flat=flat_for(case, draw), copper=np.clip(copper_for(case, lp), lo, hi),
                      mean=x_mean, net=preds[k])
        best = w.solve(draw, starts["flat"], n_plain, PLAIN).final_score / z_ed
        target = 0.99 * best
        row = dict(seed=int(s), best_ratio=best, target=target, lp_s=lp_s)
        for sname, sched, n in (("plain", PLAIN, n_plain), ("warm", WARM, n_warm)):
            for start in STARTS:
                r = w.solve(draw, starts[start], n, sched, z_ed=z_ed, stop_ratio=target,
                            check_every=check_every)
                row[f"{start}/{sname}/steps"] = int(r.steps_to_gap)
                row[f"{start}/{sname}/s"] = float(r.time_to_gap_s)
                row[f"{start}/{sname}/final"] = float(r.final_score / z_ed)
        rows[k] = row

    def lane(wi):
        for k in range(wi, len(seeds), workers):
            job(k, pool[wi])
            done[0] += 1
            if log and done[0] % 10 == 0:
                log(f"held-out days compared: {done[0]} of {len(seeds)}")

    with cf.ThreadPoolExecutor(workers) as ex:
        for f in [ex.submit(lane, i) for i in range(workers)]:
            f.result()
    for w in pool:
        w.close()
    return rows


def summarise(rows):
    """Per (start, schedule): days reaching the target, median steps and
    seconds over the days that reach it, and median seconds over all days
    with the schedule's full run time where it is not reached."""
    out = {}
    for sname in ("plain", "warm"):
        for start in STARTS:
            key = f"{start}/{sname}"
            ok = [r for r in rows if r[key + "/steps"] > 0]
            out[key] = dict(
                reached=len(ok),
                median_steps=float(np.median([r[key + "/steps"] for r in ok])) if ok else None,
                median_s=float(np.median([r[key + "/s"] for r in ok])) if ok else None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--solve-steps", type=int, default=8000)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--depth", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=20000)
    ap.add_argument("--warm-steps", type=int, default=4000)
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    case = synth.config_case(args.config)
    t0 = time.perf_counter()
    X, Y = generate(case, list(range(10000, 10000 + args.train)), args.solve_steps, log=log)
    t1 = time.perf_counter()
    log(f"training data: {args.train} days in {t1 - t0:.1f} s")
    ws = WarmStart(case, X, Y, width=args.width, depth=args.depth)
    losses = ws.train(args.train_steps)
    t2 = time.perf_counter()
    log(f"trained in {t2 - t1:.1f} s")
    rows = compare(case, ws, list(range(20000, 20000 + args.test)), n_plain=args.plain_steps,
                   n_warm=args.warm_steps, log=log)
    t3 = time.perf_counter()
    summary = dict(
        config=args.config, train_days=args.train, test_days=args.test,
        solve_steps=args.solve_steps, net=f"{X.shape[1]}-{args.width}x{args.depth}-{Y.shape[1]}",
        n_params=ws.net.n_params, data_s=t1 - t0, train_s=t2 - t1, eval_s=t3 - t2,
        train_steps=args.train_steps, loss_first=losses[0], loss_last=losses[-1],
        schedules=dict(plain=dict(PLAIN, steps=args.plain_steps),
                       warm=dict(WARM, steps=args.warm_steps)),
        by_start=summarise(rows), rows=rows)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
