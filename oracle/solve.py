"""Plain Adam loop: the Adam window of Alg. 4 (evaluate and backpropagate the
objective, contingencies included, then Alg. 3 and the clip), with the
iteration-indexed schedules of ``adam``.
"""
from __future__ import annotations

import numpy as np

from . import adam, objective

__all__ = ["class_vector", "schedule", "run"]


def class_vector(case, per_class):
    """Expand six per-class values (v, theta, p, q, r, u) to the length of x."""
    T, N, G = case.n_period, case.n_bus, case.n_gen
    lens = [T * N, T * N, T * G, T * G, T * G, T * G]
    return np.concatenate([np.full(n, float(a)) for n, a in zip(lens, per_class)])


def schedule(i, n_steps, opts):
    """(eps, beta, rho_scale, alpha[6]) at 1-based iteration i."""
    eps = adam.log_interp(opts["eps0"], opts["epsf"], i, n_steps)
    beta = adam.lin_interp(opts["beta0"], opts["betaf"], i, n_steps)
    rho = adam.lin_interp(opts["rho0"], opts["rhof"], i, n_steps)
    alpha = [adam.step_size(a0, af, i, n_steps)
             for a0, af in zip(opts["alpha0"], opts["alphaf"])]
    return eps, beta, rho, alpha


def run(model, x0, n_steps, opts, adam_cfg=None, iter0=0, m0=None, v0=None,
        record=None):
    """Run n_steps of Adam from x0; returns (x, m, v, history).

    history holds the objective total (at the schedule's eps/beta/rho) that
    each step's gradient was taken at.
    """
    case = model.case
    cfg = dict(beta1=0.9, beta2=0.999, eps=1e-8, eps_in_numerator=False)
    if adam_cfg:
        cfg.update(adam_cfg)
    lo, hi = adam.box_bounds(case)
    x = np.asarray(x0, dtype=np.float64).copy()
    m = np.zeros_like(x) if m0 is None else m0.copy()
    v = np.zeros_like(x) if v0 is None else v0.copy()
    total = opts.get("n_total", n_steps)
    hist = []
    for s in range(n_steps):
        i = iter0 + s + 1
        eps, beta, rho, alpha = schedule(i, total, opts)
        terms, g = objective.evaluate(model, x, eps, beta, rho)
        hist.append(terms["total"])
        lr = class_vector(case, alpha)
        x, m, v = adam.adam_update(x, m, v, g, i, lr, lo, hi, **cfg)
        if record is not None:
            record.append(x.copy())
    return x, m, v, hist
