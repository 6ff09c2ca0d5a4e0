"""Penalised market-surplus objective and its manual reverse pass, FP64.

The objective is the relaxed, penalised NLP of eq. (nlp_updated) with every
auxiliary variable eliminated as in Examples 1-4 of Section II-B, written for
the reduced device and network model of the synthetic grids:

    L(x; eps, beta, rho_s) = C_dev + C_bal + C_br + C_ang + C_pen + C_rsv
                             + C_ctg_max + C_ctg_mean - V_load

Basis variables x (Section II-B, Omega_c and Omega_d) are v, theta per
(period, bus) and p, q, r, u per (period, generator); u is the relaxed on/off
status in [0, 1].  Blocks are stored period-major: x = [V, TH, P, Q, R, U],
each block shaped [T, N] or [T, G].

Soft functions (footnote to Section II-C): |x|_s = sqrt(x^2 + eps^2) and
sigma(e) = sqrt(max(e, 0)^2 + eps^2); the homotopy scale beta multiplies the
power-balance, branch-flow, contingency and penalised-constraint terms
(Section II-G, "Homotopic constraint penalization").

Terms
-----
C_dev   energy cost of block bids, eq. (costs), with block size Delta_m;
        no-load cost d_t c_on u; start-up/shut-down costs on
        u_su = max(u_t - u_{t-1}, 0), u_sd = -min(u_t - u_{t-1}, 0)
        (Example 2); reserve cost d_t c_r r.  u_{-1} = u0.
C_bal   d_t beta (c_p |dp|_s + c_q |dq|_s) per (t, bus), with the mismatch of
        Example 4: dp = load + sum of from/to branch flows - generation.
C_br    d_t c_s beta sigma(max(s_fr, s_to) - s_max) per (t, branch) (Example 1).
C_ang   d_t c_ang beta sigma(|delta| - ang_max) per (t, branch), the angle
        limit of the power-flow projection (Proj. 2) used as a penalty.
C_pen   rho rho_s d_t beta sum_c sigma(a_c) over the penalised linear device
        constraints A x >= 0 of eq. (nlp_updated): headroom p + r - pmax u,
        minimum output pmin u - p, ramp up/down with start-up/shut-down
        allowances, reactive limits, reserve capability r - rmax u;
        p_{-1} = p0.
C_rsv   d_t c_rsv beta sigma(R_t - sum_j r_tj) per period.
C_ctg   per period, max_k z_tk + mean_k z_tk, with the directional contingency
        penalty of eqs. (sfr_pen)-(zctg):
        z_tk = sum_{l != k} d_t c_s beta sigma(sqrt(P_tlk^2 + qmax2_tl) - s_ctg_l),
        P_tlk the DC flow on l after branch k opens (from the balanced DC
        injections), qmax2_tl = max(q_fr^2, q_to^2) of the base-case AC flows.
V_load  constant consumer value d_t lambda_d sum_i load.

Readings of the paper fixed here (the text is silent or ambiguous):
* Branch pi-model with tap 1, no phase shift: flows of the GO3 branch model,
  consistent with the partial derivative printed in Section II-G.
* The per-period aggregation over contingencies (max plus mean) follows the
  two contingency rows of Table 1; the plain sum over k (Alg. 2 adds every
  backpropagated contingency gradient) is the alternative; the outaged
  branch itself is excluded.
* The DC injection of a bus is generation minus load; a uniform slack
  removes the period mean before the flow solve (so eq. (correction) is the
  exact gradient).
* Derivative conventions at kinks: d max(e, 0)/de = 0 at e = 0; a tie in a
  max or min takes the first argument (the from side; the smaller k in the
  argmax over contingencies; in min(p - P_cum, Delta) the p side);
  d sqrt(p^2 + q^2) := 0 at the origin; d|x|_s/dx := 0 where |x|_s = 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import network

__all__ = ["TERMS", "Model", "make_model", "unpack", "branch_flows",
           "soft_relu", "soft_relu_grad", "soft_abs", "soft_abs_grad",
           "evaluate", "ctg_excess", "ctg_term_bruteforce", "pwl_cost"]

TERMS = ("dev", "bal", "br", "ang", "pen", "rsv", "ctg_max", "ctg_mean",
         "load_value")


@dataclasses.dataclass
class Model:
    case: object
    E: np.ndarray
    y: np.ndarray
    g: np.ndarray
    b: np.ndarray
    isf: np.ndarray
    lodf: np.ndarray
    ctg: np.ndarray
    pcum: np.ndarray      # [G, M] cumulative block ends, pcum[:, m] = sum_{<=m}


def make_model(case) -> Model:
    E = network.incidence(case.n_bus, case.br_from, case.br_to)
    y = network.susceptance(case.br_r, case.br_x)
    z2 = case.br_r ** 2 + case.br_x ** 2
    g = case.br_r / z2
    b = -case.br_x / z2
    isf = network.isf_matrix(E, y, case.ref_bus)
    ctg = np.asarray(case.ctg_list, dtype=np.int64)
    lodf = network.lodf_matrix(isf, case.br_from, case.br_to, ctg)
    pcum = np.cumsum(case.gen_seg_size, axis=1)
    return Model(case=case, E=E, y=y, g=g, b=b, isf=isf, lodf=lodf, ctg=ctg,
                 pcum=pcum)


def unpack(case, x):
    T, N, G = case.n_period, case.n_bus, case.n_gen
    sl = case.block_slices()
    V = x[sl[0]].reshape(T, N)
    TH = x[sl[1]].reshape(T, N)
    P, Q, R, U = (x[s].reshape(T, G) for s in sl[2:])
    return V, TH, P, Q, R, U


def pack(case, V, TH, P, Q, R, U):
    return np.concatenate([a.reshape(-1) for a in (V, TH, P, Q, R, U)])


# --------------------------------------------------------------------------
# soft functions
# --------------------------------------------------------------------------

def soft_relu(e, eps):
    m = np.maximum(e, 0.0)
    return np.sqrt(m * m + eps * eps)


def soft_relu_grad(e, eps):
    m = np.maximum(e, 0.0)
    s = np.sqrt(m * m + eps * eps)
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.where(m > 0.0, m / np.where(s > 0.0, s, 1.0), 0.0)
    return d


def soft_abs(v, eps):
    return np.sqrt(v * v + eps * eps)


def soft_abs_grad(v, eps):
    s = np.sqrt(v * v + eps * eps)
    return np.where(s > 0.0, v / np.where(s > 0.0, s, 1.0), 0.0)


# --------------------------------------------------------------------------
# pieces of the forward model
# --------------------------------------------------------------------------

def branch_flows(model, V, TH):
    """pi-model flows (tap 1, no phase shift, charging b_ch) per (t, branch).

    p_fr = g v_f^2 + v_f v_t (-g cos d - b sin d)
    q_fr = -(b + b_ch/2) v_f^2 + v_f v_t (b cos d - g sin d)
    p_to = g v_t^2 + v_f v_t (-g cos d + b sin d)
    q_to = -(b + b_ch/2) v_t^2 + v_f v_t (b cos d + g sin d)
    with d = theta_f - theta_t.
    """
    c = model.case
    g, b, bh = model.g, model.b, 0.5 * c.br_bch
    vf = V[:, c.br_from]
    vt = V[:, c.br_to]
    d = TH[:, c.br_from] - TH[:, c.br_to]
    cs, sn = np.cos(d), np.sin(d)
    vv = vf * vt
    pf = g * vf * vf + vv * (-g * cs - b * sn)
    qf = -(b + bh) * vf * vf + vv * (b * cs - g * sn)
    pt = g * vt * vt + vv * (-g * cs + b * sn)
    qt = -(b + bh) * vt * vt + vv * (b * cs + g * sn)
    return dict(vf=vf, vt=vt, d=d, cs=cs, sn=sn, pf=pf, qf=qf, pt=pt, qt=qt)


def pwl_cost(p, seg_cost, seg_size, pcum):
    """Block-bid cost of eq. (costs) per unit time, with its derivative.

    cost = sum_m c_m max(min(p - Pcum_{m-1}, Delta_m), 0); the derivative is
    sum_m c_m [0 < p - Pcum_{m-1} <= Delta_m].
    """
    lo = np.concatenate([np.zeros(pcum.shape[:-1] + (1,)), pcum[..., :-1]], axis=-1)
    a = p[..., None] - lo
    cost = (seg_cost * np.maximum(np.minimum(a, seg_size), 0.0)).sum(axis=-1)
    dcost = (seg_cost * ((a > 0.0) & (a <= seg_size))).sum(axis=-1)
    return cost, dcost


def _device_constraints(case, P, R, U, Q):
    """The penalised device constraints a_c(x) >= 0 is feasible when a <= 0.

    Returns a list of (a [T,G], dict of partials) where partials map a
    variable name ('P', 'Pm1', 'R', 'U', 'Q') to da/dvar [T,G].  'Pm1' is the
    previous period's p (p0 for t = 0).
    """
    dt = case.dt[:, None]
    pmax, pmin = case.gen_pmax, case.gen_pmin
    one = np.ones_like(P)
    Pm1 = np.vstack([case.gen_p0[None, :], P[:-1]])
    ramp_u = dt * (case.gen_ru * U + case.gen_ru_su * (1.0 - U))
    ramp_d = dt * (case.gen_rd * U + case.gen_rd_sd * (1.0 - U))
    out = [
        (P + R - pmax * U, dict(P=one, R=one, U=-pmax * one)),
        (pmin * U - P, dict(U=pmin * one, P=-one)),
        (P - Pm1 - ramp_u, dict(P=one, Pm1=-one,
                                U=-dt * (case.gen_ru - case.gen_ru_su) * one)),
        (Pm1 - P - ramp_d, dict(Pm1=one, P=-one,
                                U=-dt * (case.gen_rd - case.gen_rd_sd) * one)),
        (Q - case.gen_qmax * U, dict(Q=one, U=-case.gen_qmax * one)),
        (case.gen_qmin * U - Q, dict(U=case.gen_qmin * one, Q=-one)),
        (R - case.gen_rmax * U, dict(R=one, U=-case.gen_rmax * one)),
    ]
    return out


def balanced_injection(case, P):
    """DC injections with uniform slack: p_bar = p_inj - mean_i p_inj [T, N]."""
    pinj = -case.load_p.copy()
    np.add.at(pinj, (slice(None), case.gen_bus), P)
    return pinj - pinj.mean(axis=1, keepdims=True)


def qmax2(fl):
    """max(q_fr^2, q_to^2) and whether the from side was taken (ties: from)."""
    qf2 = fl["qf"] ** 2
    qt2 = fl["qt"] ** 2
    use_fr = qf2 >= qt2
    return np.where(use_fr, qf2, qt2), use_fr


# --------------------------------------------------------------------------
# full evaluation
# --------------------------------------------------------------------------

def evaluate(model, x, eps, beta, rho_scale, want_grad=True, t_chunk=None, active=None,
             agg="max_mean"):
    """Objective terms (dict) and, if asked, the gradient (flat, like x).

    agg: "max_mean" (per period the worst penalty plus the mean over the K
    contingencies, Table 1's two rows) or "sum" (per period the plain sum,
    the accumulation of Alg. 2; reported in the "ctg_mean" slot, "ctg_max"
    is 0).

    active: None (every contingency is scored) or the positions (into
    model.ctg) of the contingencies scored this step, as in the contingency
    solver of Alg. 2.  A contingency outside the set takes the penalty it has
    with no overloaded branch, d_t c_s beta (L - 1) eps, a constant: it enters
    the per-period max and mean with that value and backpropagates nothing.
    """
    case = model.case
    T, N, G, L = case.n_period, case.n_bus, case.n_gen, case.n_branch
    K = model.ctg.shape[0]
    act = np.ones(K, dtype=bool)
    if active is not None:
        act = np.zeros(K, dtype=bool)
        act[np.asarray(active, dtype=np.int64)] = True
    V, TH, P, Q, R, U = unpack(case, np.asarray(x, dtype=np.float64))
    dt = case.dt
    terms = {}
    gV = np.zeros((T, N)); gTH = np.zeros((T, N))
    gP = np.zeros((T, G)); gQ = np.zeros((T, G))
    gR = np.zeros((T, G)); gU = np.zeros((T, G))

    # ---- device costs (Examples 2 and 3)
    cost, dcost = pwl_cost(P, case.gen_seg_cost, case.gen_seg_size, model.pcum)
    Um1 = np.vstack([case.gen_u0[None, :], U[:-1]])
    du = U - Um1
    usu = np.maximum(du, 0.0)
    usd = np.maximum(-du, 0.0)
    terms["dev"] = float((dt[:, None] * cost).sum()
                         + (dt[:, None] * case.gen_c_on * U).sum()
                         + (case.gen_c_su * usu).sum()
                         + (case.gen_c_sd * usd).sum()
                         + (dt[:, None] * case.gen_c_r * R).sum())
    if want_grad:
        gP += dt[:, None] * dcost
        gU += dt[:, None] * case.gen_c_on
        gR += dt[:, None] * case.gen_c_r
        dsu = case.gen_c_su * (du > 0.0)
        dsd = case.gen_c_sd * (-du > 0.0)
        gdu = dsu - dsd                       # dC/d(du)
        gU += gdu
        gU[:-1] -= gdu[1:]

    # ---- penalised device constraints
    kpen = rho_scale * case.rho * beta * dt[:, None]
    pen = 0.0
    for a, parts in _device_constraints(case, P, R, U, Q):
        pen += float((kpen * soft_relu(a, eps)).sum())
        if want_grad:
            k = kpen * soft_relu_grad(a, eps)
            for name, da in parts.items():
                if name == "P":
                    gP += k * da
                elif name == "Pm1":
                    gP[:-1] += (k * da)[1:]
                elif name == "R":
                    gR += k * da
                elif name == "U":
                    gU += k * da
                elif name == "Q":
                    gQ += k * da
    terms["pen"] = pen

    # ---- zonal reserve shortfall
    short = case.reserve_req - R.sum(axis=1)
    krs = dt * case.c_rsv * beta
    terms["rsv"] = float((krs * soft_relu(short, eps)).sum())
    if want_grad:
        gR -= (krs * soft_relu_grad(short, eps))[:, None]

    # ---- branch flows, thermal and angle penalties
    fl = branch_flows(model, V, TH)
    sf = np.hypot(fl["pf"], fl["qf"])
    st = np.hypot(fl["pt"], fl["qt"])
    use_f = sf >= st
    smax_side = np.where(use_f, sf, st)
    eb = smax_side - case.br_smax
    kbr = (dt * case.c_s * beta)[:, None]
    terms["br"] = float((kbr * soft_relu(eb, eps)).sum())
    ea = np.abs(fl["d"]) - case.ang_max
    kang = (dt * case.c_ang * beta)[:, None]
    terms["ang"] = float((kang * soft_relu(ea, eps)).sum())

    # ---- power balance (Example 4)
    dp = case.load_p.copy()
    dq = case.load_q.copy()
    np.add.at(dp, (slice(None), case.br_from), fl["pf"])
    np.add.at(dp, (slice(None), case.br_to), fl["pt"])
    np.add.at(dq, (slice(None), case.br_from), fl["qf"])
    np.add.at(dq, (slice(None), case.br_to), fl["qt"])
    np.subtract.at(dp, (slice(None), case.gen_bus), P)
    np.subtract.at(dq, (slice(None), case.gen_bus), Q)
    kb = (dt * beta)[:, None]
    terms["bal"] = float((kb * (case.c_p * soft_abs(dp, eps)
                                + case.c_q * soft_abs(dq, eps))).sum())

    # ---- contingencies
    pbar = balanced_injection(case, P)
    F = pbar @ model.isf.T                           # [T, L]
    q2, q_use_fr = qmax2(fl)
    kct = dt * case.c_s * beta                        # [T]
    z = np.zeros((T, K))
    Kidx = np.arange(K)
    sctg = case.br_smax_ctg
    chunks = range(T)
    for t in chunks:
        Pk = F[t][:, None] + model.lodf * F[t, model.ctg][None, :]   # [L, K]
        s = np.sqrt(Pk * Pk + q2[t][:, None])
        sig = soft_relu(s - sctg[:, None], eps)
        sig[model.ctg, Kidx] = 0.0
        z[t] = kct[t] * sig.sum(axis=0)
    z[:, ~act] = (kct * (L - 1) * eps)[:, None]
    kstar = np.argmax(z, axis=1) if K > 0 else np.zeros(T, dtype=np.int64)
    if agg == "sum":
        terms["ctg_max"] = 0.0
        terms["ctg_mean"] = float(z.sum())
    else:
        terms["ctg_max"] = float(z[np.arange(T), kstar].sum()) if K > 0 else 0.0
        terms["ctg_mean"] = float(z.mean(axis=1).sum()) if K > 0 else 0.0

    terms["load_value"] = float((dt[:, None] * case.load_value * case.load_p).sum())
    terms["total"] = (terms["dev"] + terms["bal"] + terms["br"] + terms["ang"]
                      + terms["pen"] + terms["rsv"] + terms["ctg_max"]
                      + terms["ctg_mean"] - terms["load_value"])
    if not want_grad:
        return terms, None

    # ---- reverse: contingencies (eqs. (2nd_lin_sys), (correction))
    Rf = np.zeros((T, L))       # dC/dF through the direct term
    Sk = np.zeros((T, K))       # dC/dF_k through the outage correction
    Qc = np.zeros((T, L))       # dC/d qmax2
    if K > 0:
        for t in chunks:
            if agg == "sum":
                w = np.where(act, 1.0, 0.0)
            else:
                w = np.where(act, 1.0 / K, 0.0)
                if act[kstar[t]]:
                    w[kstar[t]] += 1.0
            Pk = F[t][:, None] + model.lodf * F[t, model.ctg][None, :]
            s = np.sqrt(Pk * Pk + q2[t][:, None])
            ds = soft_relu_grad(s - sctg[:, None], eps)
            ds[model.ctg, Kidx] = 0.0
            inv_s = np.where(s > 0.0, 1.0 / np.where(s > 0.0, s, 1.0), 0.0)
            c = kct[t] * w[None, :] * ds                 # dC/ds
            D = c * Pk * inv_s                           # dC/dP_tlk
            Rf[t] = D.sum(axis=1)
            Sk[t] = (model.lodf * D).sum(axis=0)
            Qc[t] = (c * 0.5 * inv_s).sum(axis=1)
    Gf = Rf.copy()
    np.add.at(Gf, (slice(None), model.ctg), Sk)
    Gp = Gf @ model.isf                                  # [T, N]
    Gp -= Gp.mean(axis=1, keepdims=True)                 # eq. (correction)
    gP += Gp[:, case.gen_bus]

    # ---- reverse: balance multipliers
    lp = kb * case.c_p * soft_abs_grad(dp, eps)
    lq = kb * case.c_q * soft_abs_grad(dq, eps)
    gP -= lp[:, case.gen_bus]
    gQ -= lq[:, case.gen_bus]

    # ---- reverse: branch flows
    fr, to = case.br_from, case.br_to
    d_pf = lp[:, fr].copy(); d_pt = lp[:, to].copy()
    d_qf = lq[:, fr].copy(); d_qt = lq[:, to].copy()
    kth = kbr * soft_relu_grad(eb, eps)
    inv_sf = np.where(sf > 0.0, 1.0 / np.where(sf > 0.0, sf, 1.0), 0.0)
    inv_st = np.where(st > 0.0, 1.0 / np.where(st > 0.0, st, 1.0), 0.0)
    d_pf += np.where(use_f, kth * fl["pf"] * inv_sf, 0.0)
    d_qf += np.where(use_f, kth * fl["qf"] * inv_sf, 0.0)
    d_pt += np.where(use_f, 0.0, kth * fl["pt"] * inv_st)
    d_qt += np.where(use_f, 0.0, kth * fl["qt"] * inv_st)
    d_qf += np.where(q_use_fr, Qc * 2.0 * fl["qf"], 0.0)
    d_qt += np.where(q_use_fr, 0.0, Qc * 2.0 * fl["qt"])
    d_delta = kang * soft_relu_grad(ea, eps) * np.sign(fl["d"])

    g, b, bh = model.g, model.b, 0.5 * case.br_bch
    vf, vt, cs, sn = fl["vf"], fl["vt"], fl["cs"], fl["sn"]
    A = -g * cs - b * sn          # p_fr cross coefficient
    Bq = b * cs - g * sn          # q_fr cross coefficient
    Ct = -g * cs + b * sn         # p_to cross coefficient
    Dq = b * cs + g * sn          # q_to cross coefficient
    gvf = (d_pf * (2 * g * vf + vt * A) + d_qf * (-2 * (b + bh) * vf + vt * Bq)
           + d_pt * (vt * Ct) + d_qt * (vt * Dq))
    gvt = (d_pf * (vf * A) + d_qf * (vf * Bq)
           + d_pt * (2 * g * vt + vf * Ct) + d_qt * (-2 * (b + bh) * vt + vf * Dq))
    vv = vf * vt
    gd = (d_delta + d_pf * vv * (g * sn - b * cs) + d_qf * vv * (-b * sn - g * cs)
          + d_pt * vv * (g * sn + b * cs) + d_qt * vv * (-b * sn + g * cs))
    np.add.at(gV, (slice(None), fr), gvf)
    np.add.at(gV, (slice(None), to), gvt)
    np.add.at(gTH, (slice(None), fr), gd)
    np.subtract.at(gTH, (slice(None), to), gd)

    grad = pack(case, gV, gTH, gP, gQ, gR, gU)
    return terms, grad


def ctg_excess(model, x, eps, beta):
    """[T, K] penalty of each contingency above its no-overload value:
    d_t c_s beta sum_{l != k} (sigma(s_tlk - s_ctg_l) - eps).  A branch that is
    not overloaded adds exactly zero (sigma = eps there)."""
    case = model.case
    T = case.n_period
    V, TH, P, Q, R, U = unpack(case, np.asarray(x, dtype=np.float64))
    fl = branch_flows(model, V, TH)
    q2, _ = qmax2(fl)
    F = balanced_injection(case, P) @ model.isf.T
    K = model.ctg.shape[0]
    kct = case.dt * case.c_s * beta
    out = np.zeros((T, K))
    for t in range(T):
        Pk = F[t][:, None] + model.lodf * F[t, model.ctg][None, :]
        s = np.sqrt(Pk * Pk + q2[t][:, None])
        ex = soft_relu(s - case.br_smax_ctg[:, None], eps) - eps
        ex[model.ctg, np.arange(K)] = 0.0
        out[t] = kct[t] * ex.sum(axis=0)
    return out


def ctg_term_bruteforce(model, x, eps, beta, return_z=False):
    """C_ctg by the plain definition: one fresh DC solve per outage.

    Independent of the ISF/LODF algebra: for each contingency the network
    without that branch is re-solved (network.outage_flows).
    """
    case = model.case
    T = case.n_period
    V, TH, P, Q, R, U = unpack(case, np.asarray(x, dtype=np.float64))
    fl = branch_flows(model, V, TH)
    q2, _ = qmax2(fl)
    pbar = balanced_injection(case, P)
    K = model.ctg.shape[0]
    z = np.zeros((T, K))
    kct = case.dt * case.c_s * beta
    for ki, l_out in enumerate(model.ctg):
        f = network.outage_flows(model.E, model.y, pbar, int(l_out), case.ref_bus)
        s = np.sqrt(f * f + q2)
        sig = soft_relu(s - case.br_smax_ctg[None, :], eps)
        sig[:, l_out] = 0.0
        z[:, ki] = kct * sig.sum(axis=1)
    cmax = float(z.max(axis=1).sum()) if K else 0.0
    cmean = float(z.mean(axis=1).sum()) if K else 0.0
    if return_z:
        return cmax, cmean, z
    return cmax, cmean
