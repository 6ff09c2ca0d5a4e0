"""Copper-plate economic dispatch: the yardstick z_ed of the optimality gap.

The gap ratio of a solution is its market surplus divided by the surplus of a
relaxation that drops the network (Section III, the copper-plate bound used
for the gap figures): every device keeps its costs and constraints, power
balance is enforced for the system as a whole, and branch, angle and
contingency terms vanish.  Solved as a linear program with SciPy's HiGHS on
the host.

So that z_ed bounds the score of every point of the variable box (score =
-L at eps = 0, beta = 1, rho scale rho_f), the relaxation keeps the penalty
structure of the objective instead of hardening it:

* each penalised device constraint a_c(x) <= 0 (headroom, minimum output,
  ramping with start-up/shut-down allowances, reactive limits, reserve
  capability) gets a slack s_c >= a_c, s_c >= 0 priced at rho rho_f d_t;
* the reserve shortfall is priced at c_rsv d_t;
* the system balance keeps the price of the per-bus soft-abs penalties on a
  deficit only: summed over buses, |dp_i| >= |sum_i dp_i|, and the branch
  losses (p_fr + p_to >= 0 for r >= 0) can absorb any surplus at no cost;
* u is relaxed to [0, 1] like the solver's relaxed status, and the block
  bids are blocks 0 <= b_m <= Delta_m with convex prices, so the cheapest
  blocks fill first as in eq. (costs).

Host-only; it shares nothing with the device path.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

__all__ = ["copper_plate", "EDResult"]


class EDResult:
    """z_ed (surplus of the relaxation), its cost and the dispatch [T, G]."""

    def __init__(self, z_ed, cost, load_value, p, q, r, u, status):
        self.z_ed = z_ed
        self.cost = cost
        self.load_value = load_value
        self.p, self.q, self.r, self.u = p, q, r, u
        self.status = status


def copper_plate(case, rho_scale: float = 1.0) -> EDResult:
    """Solve the copper-plate relaxation of ``case`` (a GridCase)."""
    T, G, M = case.n_period, case.n_gen, case.n_seg
    dt = np.asarray(case.dt, dtype=np.float64)
    rho = case.rho * rho_scale
    # variable layout per (t, j): blocks b_m (M), r, u, su, sd, q, s_1..s_7;
    # then per t: reserve shortfall, p deficit, q deficit
    nv_g = M + 5 + 7
    iB, iR, iU, iSU, iSD, iQ, iS = 0, M, M + 1, M + 2, M + 3, M + 4, M + 5
    n_g = T * G * nv_g
    n = n_g + 3 * T

    def vid(t, j, off):
        return (t * G + j) * nv_g + off

    def tid(t, off):
        return n_g + 3 * t + off

    c = np.zeros(n)
    lo = np.zeros(n)
    hi = np.full(n, np.inf)
    seg_cost = np.asarray(case.gen_seg_cost, dtype=np.float64).reshape(G, M)
    seg_size = np.asarray(case.gen_seg_size, dtype=np.float64).reshape(G, M)
    for t in range(T):
        for j in range(G):
            for m in range(M):
                c[vid(t, j, iB + m)] = dt[t] * seg_cost[j, m]
                hi[vid(t, j, iB + m)] = seg_size[j, m]
            c[vid(t, j, iR)] = dt[t] * case.gen_c_r[j]
            hi[vid(t, j, iR)] = case.gen_rmax[j]
            c[vid(t, j, iU)] = dt[t] * case.gen_c_on[j]
            hi[vid(t, j, iU)] = 1.0
            c[vid(t, j, iSU)] = case.gen_c_su[j]
            c[vid(t, j, iSD)] = case.gen_c_sd[j]
            lo[vid(t, j, iQ)] = case.gen_qmin[j]
            hi[vid(t, j, iQ)] = case.gen_qmax[j]
            for q in range(7):
                c[vid(t, j, iS + q)] = rho * dt[t]
        c[tid(t, 0)] = dt[t] * case.c_rsv
        c[tid(t, 1)] = dt[t] * case.c_p
        c[tid(t, 2)] = dt[t] * case.c_q

    rows, cols, vals, rhs = [], [], [], []
    nrow = 0

    def add_row(entries, b):
        nonlocal nrow
        for col, v in entries:
            rows.append(nrow)
            cols.append(col)
            vals.append(v)
        rhs.append(b)
        nrow += 1

    for t in range(T):
        for j in range(G):
            P = [(vid(t, j, iB + m), 1.0) for m in range(M)]
            Pm1 = ([(vid(t - 1, j, iB + m), 1.0) for m in range(M)] if t > 0 else [])
            p0 = 0.0 if t > 0 else float(case.gen_p0[j])
            u = vid(t, j, iU)
            s = [vid(t, j, iS + q) for q in range(7)]
            pmax, pmin = case.gen_pmax[j], case.gen_pmin[j]
            ru, rusu = case.gen_ru[j], case.gen_ru_su[j]
            rd, rdsd = case.gen_rd[j], case.gen_rd_sd[j]
            # headroom p + r - pmax u <= s1
            add_row(P + [(vid(t, j, iR), 1.0), (u, -pmax), (s[0], -1.0)], 0.0)
            # minimum output pmin u - p <= s2
            add_row([(u, pmin)] + [(col, -1.0) for col, _ in P] + [(s[1], -1.0)], 0.0)
            # ramp up p - p_prev - dt (ru u + rusu (1 - u)) <= s3
            add_row(P + [(col, -1.0) for col, _ in Pm1]
                    + [(u, -dt[t] * (ru - rusu)), (s[2], -1.0)], dt[t] * rusu + p0)
            # ramp down p_prev - p - dt (rd u + rdsd (1 - u)) <= s4
            add_row(Pm1 + [(col, -1.0) for col, _ in P]
                    + [(u, -dt[t] * (rd - rdsd)), (s[3], -1.0)], dt[t] * rdsd - p0)
            # reactive limits q - qmax u <= s5, qmin u - q <= s6
            add_row([(vid(t, j, iQ), 1.0), (u, -case.gen_qmax[j]), (s[4], -1.0)], 0.0)
            add_row([(u, case.gen_qmin[j]), (vid(t, j, iQ), -1.0), (s[5], -1.0)], 0.0)
            # reserve capability r - rmax u <= s7
            add_row([(vid(t, j, iR), 1.0), (u, -case.gen_rmax[j]), (s[6], -1.0)], 0.0)
            # start-up and shut-down: su >= u - u_prev, sd >= u_prev - u
            u_prev = vid(t - 1, j, iU) if t > 0 else None
            u0 = 0.0 if t > 0 else float(case.gen_u0[j])
            e = [(u, 1.0), (vid(t, j, iSU), -1.0)] + ([(u_prev, -1.0)] if u_prev is not None else [])
            add_row(e, u0)
            e = [(u, -1.0), (vid(t, j, iSD), -1.0)] + ([(u_prev, 1.0)] if u_prev is not None else [])
            add_row(e, -u0)
        # reserve: R_t - sum r <= shortfall
        add_row([(vid(t, j, iR), -1.0) for j in range(G)] + [(tid(t, 0), -1.0)],
                -float(case.reserve_req[t]))
        # system balance deficits: sum load - sum gen <= deficit
        add_row([(vid(t, j, iB + m), -1.0) for j in range(G) for m in range(M)]
                + [(tid(t, 1), -1.0)], -float(np.sum(case.load_p[t])))
        add_row([(vid(t, j, iQ), -1.0) for j in range(G)] + [(tid(t, 2), -1.0)],
                -float(np.sum(case.load_q[t])))

    A = sp.csr_matrix((vals, (rows, cols)), shape=(nrow, n))
    res = linprog(c, A_ub=A, b_ub=np.asarray(rhs), bounds=np.column_stack([lo, hi]),
                  method="highs")
    if res.status != 0:
        raise RuntimeError(f"copper-plate LP failed: {res.message}")
    xg = res.x[:n_g].reshape(T, G, nv_g)
    p = xg[:, :, iB:iB + M].sum(axis=2)
    load_value = float((dt[:, None] * case.load_value * case.load_p).sum())
    return EDResult(z_ed=load_value - res.fun, cost=res.fun, load_value=load_value,
                    p=p, q=xg[:, :, iQ], r=xg[:, :, iR], u=xg[:, :, iU], status=res.status)
