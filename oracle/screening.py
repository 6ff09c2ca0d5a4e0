"""Contingency screening of the contingency solver (Alg. 2), FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Alg. 2 scores, in each Adam iteration, a worst set K_t (the top fraction of a
running list of the most severe contingencies) together with a stochastic set
S_t drawn from the rest, and backpropagates the ones whose score exceeds a
threshold zeta (Section II-F, "Contingency backpropagation summary").

Readings fixed here (the text leaves them open):
* Severity of contingency k is its largest penalty above the no-overload
  value over the periods: sev_k = max_t (z_tk - d_t c_s beta (L - 1) eps)
  (objective.ctg_excess).  A contingency that overloads nothing has severity
  exactly zero.
* The running list is refreshed by an exact step (every contingency scored)
  every R steps; the R - 1 steps between use the set chosen from it.  One set
  serves all periods (the union of the per-period sets), so that one column
  of outage factors serves every period.
* zeta applies to the worst set: only contingencies with sev_k > zeta are
  eligible for it.  Inside the scored set, backpropagation is skipped for
  every (period, branch) pair without an overload, and a contingency without
  any overload contributes exactly zero gradient, so the threshold at the
  no-overload value is part of every step.
* Set sizes are fixed: n_top = ceil(top_frac K) worst slots and
  n_act = min(K, n_top + ceil(rand_frac K)) in all; when fewer than n_top
  contingencies are eligible the random draw fills the rest.
* Worst set: eligible contingencies in order of decreasing severity, the
  smaller index first on ties.  Random set: the n_act - |worst| remaining
  contingencies with the smallest keys key(seed, r, k) (the smaller k first
  on equal keys), r the index of the refresh: a uniform draw without
  replacement, fresh at each refresh.
* key(seed, r, k) is output number r 2^32 + k + 1 of the SplitMix64 generator
  seeded with seed (Steele, Lea and Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014): state = seed + gamma n (mod 2^64), then
  the generator's mixing function.
"""
from __future__ import annotations

import math

import numpy as np

from . import adam, objective, solve

__all__ = ["GAMMA", "splitmix64_mix", "key", "counts", "severity", "select", "run"]

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64_mix(z):
    """SplitMix64's output function of the (already advanced) state z."""
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def key(seed, r, k):
    """Output r 2^32 + k + 1 of SplitMix64 seeded with seed."""
    n = (r << 32) + k + 1
    return splitmix64_mix((seed + GAMMA * n) & MASK)


def counts(K, top_frac, rand_frac):
    """(n_top, n_act) for K contingencies."""
    n_top = min(K, math.ceil(top_frac * K))
    n_act = min(K, n_top + math.ceil(rand_frac * K))
    return n_top, n_act


def severity(model, x, eps, beta):
    """sev_k = max over periods of the penalty above the no-overload value."""
    ex = objective.ctg_excess(model, x, eps, beta)
    return ex.max(axis=0) if ex.shape[1] else np.zeros(0)


def select(sev, n_top, n_act, zeta, seed, r):
    """Sorted positions of the scored contingencies after refresh r."""
    K = len(sev)
    eligible = [k for k in range(K) if sev[k] > zeta]
    worst = sorted(eligible, key=lambda k: (-sev[k], k))[:n_top]
    chosen = set(worst)
    rest = [k for k in range(K) if k not in chosen]
    drawn = sorted(rest, key=lambda k: (key(seed, r, k), k))[:n_act - len(worst)]
    return np.array(sorted(chosen.union(drawn)), dtype=np.int64)


def run(model, x0, n_steps, opts, screen, adam_cfg=None, iter0=0, m0=None, v0=None,
        active0=None, record=None):
    """solve.run with Alg. 2 screening; returns (x, m, v, history, sets).

    screen: dict(top_frac, rand_frac, zeta, refresh, seed).  Step i (1-based)
    is an exact step when (i - 1) is a multiple of refresh, or when no set has
    been chosen yet (active0 None at the first step); the set chosen from its
    severities (refresh index (i - 1) // refresh) serves the steps after it.
    sets lists (i, set) for every refresh.
    """
    case = model.case
    cfg = dict(beta1=0.9, beta2=0.999, eps=1e-8, eps_in_numerator=False)
    if adam_cfg:
        cfg.update(adam_cfg)
    lo, hi = adam.box_bounds(case)
    K = model.ctg.shape[0]
    n_top, n_act = counts(K, screen["top_frac"], screen["rand_frac"])
    R = screen["refresh"]
    x = np.asarray(x0, dtype=np.float64).copy()
    m = np.zeros_like(x) if m0 is None else m0.copy()
    v = np.zeros_like(x) if v0 is None else v0.copy()
    total = opts.get("n_total", n_steps)
    active = None if active0 is None else np.asarray(active0, dtype=np.int64)
    hist, sets = [], []
    for s in range(n_steps):
        i = iter0 + s + 1
        eps, beta, rho, alpha = solve.schedule(i, total, opts)
        if (i - 1) % R == 0 or active is None:
            terms, g = objective.evaluate(model, x, eps, beta, rho)
            sev = severity(model, x, eps, beta)
            active = select(sev, n_top, n_act, screen["zeta"], screen["seed"], (i - 1) // R)
            sets.append((i, active.copy()))
        else:
            terms, g = objective.evaluate(model, x, eps, beta, rho, active=active)
        hist.append(terms["total"])
        x, m, v = adam.adam_update(x, m, v, g, i, solve.class_vector(case, alpha), lo, hi, **cfg)
        if record is not None:
            record.append((x.copy(), m.copy(), v.copy(), active.copy()))
    return x, m, v, hist, sets
