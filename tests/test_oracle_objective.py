"""Pins of the oracle's objective and manual reverse pass (Section II)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import adam, network, objective as ob
from paper_2310_06650_amd import synth
from tests._cases import tiny_case

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- branch model

def test_flat_start_has_no_flow():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    V = np.ones((1, c.n_bus))
    TH = np.zeros((1, c.n_bus))
    fl = ob.branch_flows(m, V, TH)
    for k in ("pf", "qf", "pt", "qt"):
        assert np.abs(fl[k]).max() < 1e-12


def test_printed_partial_dpfr_dvto():
    """Section II-G prints d p_fr / d v_to = (-g cos d - b sin d) v_fr / tau."""
    c = synth.config_case("c1")
    m = ob.make_model(c)
    rng = np.random.default_rng(2)
    V = rng.uniform(0.9, 1.1, size=(1, c.n_bus))
    TH = rng.normal(0, 0.2, size=(1, c.n_bus))
    fl = ob.branch_flows(m, V, TH)
    printed = (-m.g * np.cos(fl["d"]) - m.b * np.sin(fl["d"])) * fl["vf"]
    for l in range(c.n_branch):
        j = c.br_to[l]
        h = 1e-6
        Vp = V.copy(); Vp[0, j] += h
        Vm = V.copy(); Vm[0, j] -= h
        fd = (ob.branch_flows(m, Vp, TH)["pf"][0, l]
              - ob.branch_flows(m, Vm, TH)["pf"][0, l]) / (2 * h)
        assert abs(fd - printed[0, l]) < 1e-7 * max(1.0, abs(printed[0, l]))


def test_losses_nonnegative():
    c = synth.config_case("c2")
    m = ob.make_model(c)
    rng = np.random.default_rng(4)
    V = rng.uniform(0.9, 1.1, size=(3, c.n_bus))
    TH = rng.normal(0, 0.3, size=(3, c.n_bus))
    fl = ob.branch_flows(m, V, TH)
    assert (fl["pf"] + fl["pt"] >= -1e-12).all()


# ---------------------------------------------------------------- devices

def test_pwl_cost_equals_block_fill():
    """eq. (costs) against filling the blocks one by one."""
    rng = np.random.default_rng(0)
    size = rng.uniform(0.2, 1.0, size=(50, 3))
    cost = np.sort(rng.uniform(1, 10, size=(50, 3)), axis=1)
    pcum = np.cumsum(size, axis=1)
    p = rng.uniform(0, 1, size=50) * pcum[:, -1]
    got, _ = ob.pwl_cost(p, cost, size, pcum)
    for j in range(50):
        rem, acc = p[j], 0.0
        for mm in range(3):
            take = min(rem, size[j, mm])
            acc += cost[j, mm] * take
            rem -= take
        assert abs(acc - got[j]) < 1e-12 * max(1.0, acc)


def test_device_cost_hand_example():
    gd = _gold("device_2x3.json")
    c = tiny_case(2, [0], [1], [0.1], [0, 1], T=3, dt=gd["dt"],
                  seg_size=gd["seg_size"], seg_cost=gd["seg_cost"],
                  gen_c_on=np.array(gd["c_on"]), gen_c_su=np.array(gd["c_su"]),
                  gen_c_sd=np.array(gd["c_sd"]), gen_c_r=np.array(gd["c_r"]),
                  gen_u0=np.array(gd["u0"]))
    m = ob.make_model(c)
    V = np.ones((3, 2)); TH = np.zeros((3, 2))
    P = np.array(gd["P"]); U = np.array(gd["U"]); R = np.array(gd["R"])
    x = ob.pack(c, V, TH, P, np.zeros((3, 2)), R, U)
    terms, _ = ob.evaluate(m, x, 1e-3, 1.0, 1.0, want_grad=False)
    assert abs(terms["dev"] - gd["total"]) < 1e-12
    e, _ = ob.pwl_cost(P, c.gen_seg_cost, c.gen_seg_size, m.pcum)
    assert abs((np.array(gd["dt"])[:, None] * e).sum() - gd["energy"]) < 1e-12


# ---------------------------------------------------------------- derivatives

def _fd_check_classes(m, x, eps, beta, rho, n_per_class, seed, tol, h_rel=1e-6):
    case = m.case
    terms, g = ob.evaluate(m, x, eps, beta, rho)
    rng = np.random.default_rng(seed)
    for s in case.block_slices():
        idx = rng.choice(np.arange(s.start, s.stop), size=min(n_per_class, s.stop - s.start),
                         replace=False)
        fd = np.empty(len(idx))
        for a, j in enumerate(idx):
            h = h_rel * max(1.0, abs(x[j]))
            xp = x.copy(); xp[j] += h
            xm = x.copy(); xm[j] -= h
            fp = ob.evaluate(m, xp, eps, beta, rho, want_grad=False)[0]
            fm = ob.evaluate(m, xm, eps, beta, rho, want_grad=False)[0]
            # difference term by term: the large totals cancel less accurately
            fd[a] = sum((fp[k] - fm[k]) for k in ob.TERMS if k != "load_value") / (2 * h)
        err = np.abs(fd - g[idx]).max() / max(np.abs(g[s]).max(), 1e-30)
        assert err < tol, (s, err)
    return terms, g


@pytest.mark.parametrize("seed", [7, 8])
def test_gradient_matches_central_differences_c1(seed):
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, seed)
    _fd_check_classes(m, x, 0.05, 0.7, 0.8, 40, seed, 2e-7)


def test_gradient_matches_central_differences_c2_sampled():
    c = synth.config_case("c2")
    m = ob.make_model(c)
    x = synth.random_point(c, 21, spread=0.3)
    _fd_check_classes(m, x, 0.05, 1.0, 1.0, 4, 3, 1e-5)


def test_angle_shift_invariance():
    """L depends on angle differences only, so sum_i dL/dtheta_ti = 0."""
    c = synth.config_case("c2")
    m = ob.make_model(c)
    x = synth.random_point(c, 5)
    _, g = ob.evaluate(m, x, 0.01, 1.0, 1.0)
    sl = c.block_slices()
    gth = g[sl[1]].reshape(c.n_period, c.n_bus)
    assert np.abs(gth.sum(axis=1)).max() < 1e-9 * np.abs(gth).max() * c.n_bus


def test_uniform_slack_makes_ctg_term_blind_to_uniform_shift():
    """With the uniform slack (eq. (correction)) a load change spread evenly
    over all buses leaves every contingency flow unchanged."""
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 2)
    t0, _ = ob.evaluate(m, x, 0.01, 1.0, 1.0, want_grad=False)
    c.load_p = c.load_p + 0.37
    t1, _ = ob.evaluate(m, x, 0.01, 1.0, 1.0, want_grad=False)
    assert abs(t0["ctg_max"] - t1["ctg_max"]) < 1e-9 * abs(t0["ctg_max"])
    assert abs(t0["ctg_mean"] - t1["ctg_mean"]) < 1e-9 * abs(t0["ctg_mean"])


def test_ctg_gradient_of_injections_sums_to_zero():
    """eq. (correction): with a generator at every bus, moving all of them by
    the same amount shifts every injection uniformly, which the uniform slack
    absorbs, so the contingency gradient over generators sums to zero."""
    n = 5
    c = tiny_case(n, [0, 1, 2, 3, 4, 0], [1, 2, 3, 4, 0, 2],
                  [0.1, 0.2, 0.15, 0.1, 0.12, 0.3], list(range(n)), T=2,
                  br_r=[0.01] * 6, ctg=[0, 1, 2, 3, 4, 5])
    c.c_p = c.c_q = c.c_ang = c.c_rsv = c.rho = 0.0
    c.gen_c_on[:] = 0; c.gen_c_su[:] = 0; c.gen_c_sd[:] = 0; c.gen_c_r[:] = 0
    c.gen_seg_cost[:] = 0
    c.br_smax[:] = 1e6
    c.br_smax_ctg[:] = 0.05
    m = ob.make_model(c)
    x = synth.random_point(c, 9)
    _, g = ob.evaluate(m, x, 0.01, 1.0, 1.0)
    gp = g[c.block_slices()[2]].reshape(c.n_period, c.n_gen)
    assert np.abs(gp).max() > 1.0
    assert np.abs(gp.sum(axis=1)).max() < 1e-12 * np.abs(gp).max() * n


def test_ctg_all_overloaded_matches_bruteforce():
    """Every branch overloaded in every outage: the LODF form still equals the
    per-outage re-solve, so both leave the outaged branch out the same way."""
    c = tiny_case(3, [0, 1, 0], [1, 2, 2], [0.1, 0.2, 0.15], [0, 2], T=2,
                  br_r=[0.01, 0.02, 0.01], ctg=[0, 1, 2])
    c.br_smax_ctg[:] = 1e-3
    m = ob.make_model(c)
    x = synth.random_point(c, 3)
    t, _ = ob.evaluate(m, x, 0.0, 1.0, 1.0, want_grad=False)
    cmax, cmean = ob.ctg_term_bruteforce(m, x, 0.0, 1.0)
    assert abs(t["ctg_max"] - cmax) < 1e-12 * cmax
    assert abs(t["ctg_mean"] - cmean) < 1e-12 * cmean


# ---------------------------------------------------------------- contingencies

def test_ctg_lodf_form_equals_bruteforce_c1():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    for seed in (1, 2, 3):
        x = synth.random_point(c, seed)
        terms, _ = ob.evaluate(m, x, 0.02, 0.9, 1.0, want_grad=False)
        cmax, cmean = ob.ctg_term_bruteforce(m, x, 0.02, 0.9)
        assert abs(terms["ctg_max"] - cmax) < 1e-10 * abs(cmax)
        assert abs(terms["ctg_mean"] - cmean) < 1e-10 * abs(cmean)


def test_ctg_lodf_form_equals_bruteforce_c2_subset():
    c = synth.config_case("c2")
    c.ctg_list = c.ctg_list[::40].copy()
    m = ob.make_model(c)
    x = synth.random_point(c, 4, spread=0.3)
    terms, _ = ob.evaluate(m, x, 0.02, 1.0, 1.0, want_grad=False)
    cmax, cmean = ob.ctg_term_bruteforce(m, x, 0.02, 1.0)
    assert abs(terms["ctg_max"] - cmax) < 1e-9 * abs(cmax)
    assert abs(terms["ctg_mean"] - cmean) < 1e-9 * abs(cmean)


# ---------------------------------------------------------------- Adam

def test_schedule_golden_values():
    gd = _gold("schedule.json")
    n = 1000
    for th, s in zip(gd["t_hat"], gd["scale"]):
        i = (th + 1.0) / 2.0 * n
        assert abs(adam.sched_scale(i, n) - s) < 1e-15
    # alpha at the midpoint: alpha0 * (alphaf/alpha0)^0.625
    a = adam.step_size(1e-2, 1e-5, 500, 1000)
    assert abs(a - 1e-2 * 10 ** (0.625 * -3.0)) < 1e-17


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    g = rng.normal(size=100) * 10.0 ** rng.integers(-6, 6, size=100)
    x0 = np.zeros(100)
    lo, hi = np.full(100, -np.inf), np.full(100, np.inf)
    x, _, _ = adam.adam_update(x0, np.zeros(100), np.zeros(100), g, 1, 0.5, lo, hi)
    np.testing.assert_allclose(x, -0.5 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    x, _, _ = adam.adam_update(x0, np.zeros(100), np.zeros(100), g, 1, 0.5, lo, hi,
                               eps_in_numerator=True)
    np.testing.assert_allclose(x, -0.5 * (g + 1e-8) / (np.abs(g) + 1e-8), rtol=1e-12)
    # clip (Alg. 3, last step)
    x, _, _ = adam.adam_update(x0, np.zeros(100), np.zeros(100), g, 1, 0.5,
                               np.full(100, -0.1), np.full(100, 0.2))
    assert x.min() >= -0.1 and x.max() <= 0.2


def test_adam_second_step_closed_form():
    g1, g2 = 3.0, -1.0
    b1, b2, e = 0.9, 0.999, 1e-8
    x = np.zeros(1); m = np.zeros(1); v = np.zeros(1)
    inf = np.array([np.inf])
    x, m, v = adam.adam_update(x, m, v, np.array([g1]), 1, 1.0, -inf, inf)
    x, m, v = adam.adam_update(x, m, v, np.array([g2]), 2, 1.0, -inf, inf)
    m2 = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    v2 = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    step1 = g1 / (abs(g1) + e)
    assert abs(x[0] - (-step1 - m2 / (math.sqrt(v2) + e))) < 1e-14


def test_oracle_adam_decreases_objective_c1():
    from oracle import solve
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x0 = synth.flat_start(c)
    opts = dict(eps0=1e-2, epsf=1e-2, beta0=1.0, betaf=1.0, rho0=1.0, rhof=1.0,
                alpha0=[1e-3] * 6, alphaf=[1e-3] * 6)
    x, _, _, hist = solve.run(m, x0, 200, opts)
    assert hist[-1] < hist[0]


# ---------------------------------------------------------------- special cases

def _one_gen_case(T=2):
    # 2 buses, 1 branch, one generator at bus 0; loads only at bus 0
    c = tiny_case(2, [0], [1], [0.1], [0], T=T, seg_size=[[1.0, 1.0, 1.0]])
    c.load_p = np.zeros((T, 2)); c.load_p[:, 0] = 1.2
    c.load_q = np.zeros((T, 2)); c.load_q[:, 0] = 0.3
    c.reserve_req = np.full(T, 0.1)
    c.gen_p0 = np.array([1.2])
    return c


def _x(c, P, Q, R, U, V=None, TH=None):
    T, N = c.n_period, c.n_bus
    V = np.ones((T, N)) if V is None else V
    TH = np.zeros((T, N)) if TH is None else TH
    f = lambda a: np.asarray(a, dtype=float).reshape(T, c.n_gen)
    return ob.pack(c, V, TH, f(P), f(Q), f(R), f(U))


def test_floors_when_everything_is_satisfied():
    """Flat voltages carry no flow; a generator meeting its own bus load and
    all limits leaves only the soft-function floors: eps per soft term."""
    c = _one_gen_case()
    m = ob.make_model(c)
    x = _x(c, [1.2, 1.2], [0.3, 0.3], [0.15, 0.15], [1.0, 1.0])
    eps, beta, rs = 1e-3, 0.5, 0.25
    t, _ = ob.evaluate(m, x, eps, beta, rs, want_grad=False)
    dsum = c.dt.sum()
    assert abs(t["bal"] - dsum * beta * (c.c_p + c.c_q) * eps * c.n_bus) < 1e-12
    assert abs(t["pen"] - rs * c.rho * beta * eps * 7 * dsum) < 1e-12
    assert abs(t["rsv"] - c.c_rsv * beta * eps * dsum) < 1e-12
    assert abs(t["br"] - c.c_s * beta * eps * dsum) < 1e-12
    assert abs(t["ang"] - c.c_ang * beta * eps * dsum) < 1e-12


@pytest.mark.parametrize("which", ["headroom", "mingen", "rampup", "rampdown",
                                   "qmax", "qmin", "rcap"])
def test_single_violation_exact(which):
    """At eps = 0 the penalty is rho * d_t * beta * (violation) for the one
    violated device constraint."""
    c = _one_gen_case(T=2)
    c.dt = np.array([1.0, 0.5])
    m = ob.make_model(c)
    pmax, pmin = c.gen_pmax[0], c.gen_pmin[0]
    ru, rsu = c.gen_ru[0], c.gen_ru_su[0]
    P = [1.2, 1.2]; Q = [0.3, 0.3]; R = [0.1, 0.1]; U = [1.0, 1.0]
    viol = 0.05
    t_v = 1
    if which == "headroom":
        R = [0.1, pmax - 1.2 + viol]
        c.gen_rmax[:] = 5.0
    elif which == "mingen":
        U = [1.0, 0.6]; P = [1.2, 0.6 * pmin - viol]
        # keep the ramp-down limit loose and reserve capability satisfied
        c.gen_rd[:] = 10.0; c.gen_rd_sd[:] = 10.0
        R = [0.1, 0.0]
    elif which == "rampup":
        P = [1.2, 1.2 + 0.5 * ru + viol]
        c.reserve_req[:] = 0.0; R = [0.0, 0.0]
    elif which == "rampdown":
        c.gen_rd[:] = 0.4; c.gen_rd_sd[:] = 0.3
        P = [1.2, 1.2 - 0.5 * 0.4 - viol]
    elif which == "qmax":
        Q = [0.3, c.gen_qmax[0] + viol]
    elif which == "qmin":
        Q = [0.3, c.gen_qmin[0] - viol]
    elif which == "rcap":
        c.reserve_req[:] = 0.0
        R = [0.0, c.gen_rmax[0] + viol]
    x = _x(c, P, Q, R, U)
    beta, rs = 0.8, 0.5
    t, _ = ob.evaluate(m, x, 0.0, beta, rs, want_grad=False)
    want = rs * c.rho * beta * c.dt[t_v] * viol
    assert abs(t["pen"] - want) < 1e-9 * want, (which, t["pen"], want)


def test_reserve_shortfall_exact():
    c = _one_gen_case(T=2)
    c.dt = np.array([1.0, 2.0])
    m = ob.make_model(c)
    x = _x(c, [1.2, 1.2], [0.3, 0.3], [0.1, 0.04], [1.0, 1.0])
    t, _ = ob.evaluate(m, x, 0.0, 0.7, 1.0, want_grad=False)
    assert abs(t["rsv"] - 2.0 * c.c_rsv * 0.7 * 0.06) < 1e-9


def test_balance_with_zero_flows_exact():
    """Flat voltages: the mismatch is load minus generation at each bus
    (Example 4 with no branch flow)."""
    c = _one_gen_case(T=1)
    c.load_p[0, 1] = 0.25
    m = ob.make_model(c)
    x = _x(c, [1.0], [0.1], [0.1], [1.0])
    t, _ = ob.evaluate(m, x, 0.0, 1.0, 1.0, want_grad=False)
    want = c.c_p * (0.2 + 0.25) + c.c_q * 0.2
    assert abs(t["bal"] - want) < 1e-9 * want


def test_thermal_and_angle_exact_two_bus():
    """One lossless branch at unit voltages: p_fr = -b sin d = sin(d)/x and
    q_fr = q_to = (1 - cos d)/x, so s = sqrt(2(1 - cos d))/x = 2 sin(d/2)/x."""
    c = _one_gen_case(T=1)
    c.br_smax[:] = 1.0
    c.ang_max = 0.3
    m = ob.make_model(c)
    d = 0.4
    x = _x(c, [1.2], [0.3], [0.1], [1.0], TH=np.array([[d, 0.0]]))
    t, _ = ob.evaluate(m, x, 0.0, 1.0, 1.0, want_grad=False)
    s = 2.0 * math.sin(d / 2) / 0.1
    assert abs(t["br"] - c.c_s * (s - 1.0)) < 1e-9 * c.c_s
    assert abs(t["ang"] - c.c_ang * (d - 0.3)) < 1e-9 * c.c_ang


# ---------------------------------------------------------------- sum aggregation

def test_sum_aggregation_is_k_times_the_mean_and_matches_bruteforce():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 3)
    K = len(m.ctg)
    ts, _ = ob.evaluate(m, x, 0.02, 0.9, 1.0, want_grad=False, agg="sum")
    tm, _ = ob.evaluate(m, x, 0.02, 0.9, 1.0, want_grad=False)
    assert ts["ctg_max"] == 0.0
    assert abs(ts["ctg_mean"] - K * tm["ctg_mean"]) <= 1e-12 * ts["ctg_mean"]
    _, _, zb = ob.ctg_term_bruteforce(m, x, 0.02, 0.9, return_z=True)
    assert abs(ts["ctg_mean"] - zb.sum()) <= 1e-10 * ts["ctg_mean"]
    for k in ob.TERMS:
        if k not in ("ctg_max", "ctg_mean"):
            assert ts[k] == tm[k]


def test_sum_aggregation_gradient_matches_central_differences():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 5)
    eps, beta, rho = 0.05, 0.7, 0.8
    _, g = ob.evaluate(m, x, eps, beta, rho, agg="sum")
    rng = np.random.default_rng(4)
    for s in c.block_slices()[:4]:
        idx = rng.choice(np.arange(s.start, s.stop), size=12, replace=False)
        fd = []
        for j in idx:
            h = 1e-6 * max(1.0, abs(x[j]))
            xp = x.copy(); xp[j] += h
            xm = x.copy(); xm[j] -= h
            fp = ob.evaluate(m, xp, eps, beta, rho, want_grad=False, agg="sum")[0]
            fm = ob.evaluate(m, xm, eps, beta, rho, want_grad=False, agg="sum")[0]
            fd.append(sum(fp[k] - fm[k] for k in ob.TERMS if k != "load_value") / (2 * h))
        err = np.abs(np.array(fd) - g[idx]).max() / max(np.abs(g[s]).max(), 1e-30)
        assert err < 2e-7, (s, err)
