"""Step-size schedule and the modified Adam update (Section II-G, Alg. 3).

Schedule, eqs. (norm_t)-(step_size): with t_hat = 2 (t - t0)/(tf - t0) - 1,
the magnitude scale is s = e^{4 t_hat} / (0.6 + e^{4 t_hat}) and the step is
alpha = alpha0 * 10^(s * log10(alpha_f / alpha0)).  The paper indexes t by
wall-clock time; this oracle indexes it by the Adam iteration i (t0 = 0,
tf = number of steps), which makes runs reproducible.  The soft-function
width eps follows the same curve between its own end points ("decays in the
same fashion ... over more orders of magnitude"), and the homotopy scale
beta and the penalty scale rho grow linearly (Section II-G, "Homotopic
constraint penalization").

Adam (Alg. 3): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2; then
x <- x - alpha (m/(1-b1^i) + e_n) / (sqrt(v/(1-b2^i)) + e), followed by a clip
to the box.  The paper prints e in the numerator as well (e_n = e); the
standard update of Kingma and Ba, which the paper cites, has e_n = 0.  Both
forms are provided; the standard one is the default.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["sched_scale", "step_size", "log_interp", "lin_interp",
           "adam_update", "box_bounds"]


def sched_scale(i, n_steps, t0=0.0):
    """Magnitude scale of eq. (mag_scale) at iteration i of n_steps."""
    that = 2.0 * (i - t0) / (n_steps - t0) - 1.0
    e = math.exp(4.0 * that)
    return e / (0.6 + e)


def step_size(alpha0, alphaf, i, n_steps):
    """Eq. (step_size) with the iteration-indexed scale."""
    s = sched_scale(i, n_steps)
    return alpha0 * 10.0 ** (s * math.log10(alphaf / alpha0))


def log_interp(v0, vf, i, n_steps):
    """The same reflected-sigmoid curve between two positive end points."""
    return step_size(v0, vf, i, n_steps)


def lin_interp(v0, vf, i, n_steps):
    return v0 + (vf - v0) * (i / n_steps)


def box_bounds(case):
    """Lower/upper bound per entry of x (theta unbounded)."""
    T, N, G = case.n_period, case.n_bus, case.n_gen
    inf = np.inf
    lo = np.concatenate([
        np.tile(case.v_min, T), np.full(T * N, -inf),
        np.zeros(T * G), np.tile(case.gen_qmin, T), np.zeros(T * G),
        np.zeros(T * G)])
    hi = np.concatenate([
        np.tile(case.v_max, T), np.full(T * N, inf),
        np.tile(case.gen_pmax, T), np.tile(case.gen_qmax, T),
        np.tile(case.gen_rmax, T), np.ones(T * G)])
    return lo, hi


def adam_update(x, m, v, g, i, lr, lo, hi, beta1=0.9, beta2=0.999, eps=1e-8,
                eps_in_numerator=False):
    """One modified-Adam step (Alg. 3) on copies; returns (x, m, v).

    lr is a per-entry step size (broadcastable to x); i is 1-based.
    """
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** i)
    vh = v / (1.0 - beta2 ** i)
    num = mh + eps if eps_in_numerator else mh
    x = x - lr * num / (np.sqrt(vh) + eps)
    x = np.minimum(np.maximum(x, lo), hi)
    return x, m, v
