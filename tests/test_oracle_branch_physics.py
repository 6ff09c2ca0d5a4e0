"""Independent pins of the oracle's AC branch physics (Section II-B, Example 1
and Example 4; Section II-G partials) on lossy branches with line charging.

The reference values here come from complex phasor arithmetic written in the
tests themselves, not from the oracle's real-valued pi-model:

* branch currents  I_fr = y_s (V_f - V_t) + j (b_ch / 2) V_f,
                   I_to = y_s (V_t - V_f) + j (b_ch / 2) V_t,
  with the series admittance y_s = 1 / (r + j x) and phasors V = v e^{j theta};
* complex power leaving each end S = V conj(I);
* bus injections S_i = V_i conj((Y_bus V)_i) from an admittance matrix the
  test assembles branch by branch;
* post-outage DC flows from a fresh Laplacian solve per removed branch.

A sign slip in the oracle's flows (for instance in the g sin(delta) parts of
the reactive flows) or in the way flows enter the bus mismatch makes one of
these fail.
"""
import math

import numpy as np
import pytest

from oracle import objective as ob
from tests._cases import tiny_case

MESH4 = dict(n_bus=4, br_from=[0, 1, 2, 3, 0], br_to=[1, 2, 3, 0, 2])


def _lossy_case(n_bus, br_from, br_to, T, seed, gen_bus=None, **over):
    rng = np.random.default_rng(seed)
    L = len(br_from)
    x = rng.uniform(0.05, 0.2, size=L)
    r = x * rng.uniform(0.1, 0.4, size=L)
    over.setdefault("br_bch", rng.uniform(0.01, 0.1, size=L))
    gen_bus = list(range(n_bus)) if gen_bus is None else gen_bus
    return tiny_case(n_bus, br_from, br_to, x, gen_bus, T=T, br_r=r, **over)


def _phasors(rng, T, N):
    v = rng.uniform(0.92, 1.08, size=(T, N))
    th = rng.normal(0.0, 0.15, size=(T, N))
    return v, th, v * np.exp(1j * th)


def _branch_power(c, Vc):
    """Complex power leaving the from and to ends of every branch [T, L]."""
    ys = 1.0 / (c.br_r + 1j * c.br_x)
    jb = 0.5j * c.br_bch
    Vf = Vc[:, c.br_from]
    Vt = Vc[:, c.br_to]
    S_fr = Vf * np.conj(ys * (Vf - Vt) + jb * Vf)
    S_to = Vt * np.conj(ys * (Vt - Vf) + jb * Vt)
    return S_fr, S_to


def _ybus(c):
    N = c.n_bus
    Y = np.zeros((N, N), dtype=complex)
    for l in range(c.n_branch):
        f, t = int(c.br_from[l]), int(c.br_to[l])
        ys = 1.0 / (c.br_r[l] + 1j * c.br_x[l])
        sh = 0.5j * c.br_bch[l]
        Y[f, f] += ys + sh
        Y[t, t] += ys + sh
        Y[f, t] -= ys
        Y[t, f] -= ys
    return Y


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pi_model_flows_equal_complex_power(seed):
    """p, q at both ends of lossy, charged branches equal Re and Im of
    V conj(I) with the pi-model currents."""
    c = _lossy_case(**MESH4, T=3, seed=seed)
    m = ob.make_model(c)
    rng = np.random.default_rng(100 + seed)
    v, th, Vc = _phasors(rng, c.n_period, c.n_bus)
    fl = ob.branch_flows(m, v, th)
    S_fr, S_to = _branch_power(c, Vc)
    scale = np.abs(S_fr).max()
    for name, ref in (("pf", S_fr.real), ("qf", S_fr.imag),
                      ("pt", S_to.real), ("qt", S_to.imag)):
        err = np.abs(fl[name] - ref).max() / scale
        assert err < 1e-14, (name, err)


def test_series_loss_equals_current_squared_times_r():
    """Without charging, p_fr + p_to is the series loss r |I|^2."""
    c = _lossy_case(**MESH4, T=2, seed=7, br_bch=np.zeros(5))
    m = ob.make_model(c)
    rng = np.random.default_rng(8)
    v, th, Vc = _phasors(rng, c.n_period, c.n_bus)
    fl = ob.branch_flows(m, v, th)
    I = (Vc[:, c.br_from] - Vc[:, c.br_to]) / (c.br_r + 1j * c.br_x)
    loss = c.br_r * np.abs(I) ** 2
    assert np.abs(fl["pf"] + fl["pt"] - loss).max() < 1e-14 * loss.max()
    assert (loss > 1e-6).all()


@pytest.mark.parametrize("grid", ["two_bus", "mesh4"])
def test_power_flow_consistent_point_sits_on_the_balance_floor(grid):
    """Example 4: at a point where each bus's generation minus load equals the
    complex power it injects into the network (V_i conj((Y_bus V)_i)), every
    mismatch is zero and C_bal equals its soft-abs floor d_t beta (c_p + c_q)
    eps per bus."""
    if grid == "two_bus":
        c = _lossy_case(2, [0], [1], T=2, seed=11, gen_bus=[0])
    else:
        c = _lossy_case(**MESH4, T=2, seed=12)
    T, N, G = c.n_period, c.n_bus, c.n_gen
    m = ob.make_model(c)
    rng = np.random.default_rng(13)
    v, th, Vc = _phasors(rng, T, N)
    S_inj = Vc * np.conj(Vc @ _ybus(c).T)            # [T, N]
    gen_at = np.full(N, -1)
    gen_at[c.gen_bus] = np.arange(G)
    load_p = rng.uniform(0.1, 0.4, size=(T, N))
    load_q = rng.uniform(0.0, 0.1, size=(T, N))
    P = np.zeros((T, G))
    Q = np.zeros((T, G))
    for i in range(N):
        if gen_at[i] >= 0:
            P[:, gen_at[i]] = S_inj[:, i].real + load_p[:, i]
            Q[:, gen_at[i]] = S_inj[:, i].imag + load_q[:, i]
        else:
            # a bus without generation: its load is what the network delivers
            load_p[:, i] = -S_inj[:, i].real
            load_q[:, i] = -S_inj[:, i].imag
    c.load_p = load_p
    c.load_q = load_q
    x = ob.pack(c, v, th, P, Q, np.zeros((T, G)), np.ones((T, G)))
    eps, beta = 1e-3, 0.7
    t, g = ob.evaluate(m, x, eps, beta, 1.0)
    floor = c.dt.sum() * beta * (c.c_p + c.c_q) * eps * N
    assert abs(t["bal"] - floor) < 1e-12 * floor, (t["bal"], floor)
    # the same point with every branch flow's sign reversed in the mismatch
    # (load - flows - generation) is far from the floor
    fl = ob.branch_flows(m, v, th)
    dp = load_p.copy()
    np.subtract.at(dp, (slice(None), c.br_from), fl["pf"])
    np.subtract.at(dp, (slice(None), c.br_to), fl["pt"])
    np.subtract.at(dp, (slice(None), c.gen_bus), P)
    assert np.abs(dp).max() > 1e3 * eps


def test_balance_mismatch_of_a_loaded_lossy_line():
    """Two buses, generator at bus 0 producing exactly the power the line
    takes at its sending end, load at bus 1 set to twice what the line
    delivers: at eps = 0, C_bal = c_p |p_del| + c_q |q_del| (bus 1 short by one
    delivery) and nothing at bus 0."""
    c = _lossy_case(2, [0], [1], T=1, seed=21, gen_bus=[0])
    m = ob.make_model(c)
    v = np.array([[1.03, 0.97]])
    th = np.array([[0.12, -0.05]])
    Vc = v * np.exp(1j * th)
    S_fr, S_to = _branch_power(c, Vc)
    p_del, q_del = -S_to.real[0, 0], -S_to.imag[0, 0]
    assert p_del > 0.1
    c.load_p = np.array([[0.0, 2.0 * p_del]])
    c.load_q = np.array([[0.0, 2.0 * q_del]])
    P = np.array([[S_fr.real[0, 0]]])
    Q = np.array([[S_fr.imag[0, 0]]])
    x = ob.pack(c, v, th, P, Q, np.zeros((1, 1)), np.ones((1, 1)))
    t, _ = ob.evaluate(m, x, 0.0, 1.0, 1.0, want_grad=False)
    want = c.c_p * abs(p_del) + c.c_q * abs(q_del)
    assert abs(t["bal"] - want) < 1e-12 * want, (t["bal"], want)


def test_thermal_term_of_lossy_charged_branches():
    """C_br at eps = 0: d_t c_s beta max(|S_fr|, |S_to|) - s_max summed over
    overloaded branches, with |S| from complex power."""
    c = _lossy_case(**MESH4, T=2, seed=31)
    c.dt = np.array([1.0, 0.5])
    m = ob.make_model(c)
    rng = np.random.default_rng(32)
    v, th, Vc = _phasors(rng, c.n_period, c.n_bus)
    S_fr, S_to = _branch_power(c, Vc)
    smag = np.maximum(np.abs(S_fr), np.abs(S_to))
    c.br_smax = 0.5 * smag.mean(axis=0)
    x = ob.pack(c, v, th, np.zeros((2, 4)), np.zeros((2, 4)), np.zeros((2, 4)),
                np.ones((2, 4)))
    beta = 0.6
    t, _ = ob.evaluate(m, x, 0.0, beta, 1.0, want_grad=False)
    want = (c.dt[:, None] * c.c_s * beta * np.maximum(smag - c.br_smax, 0.0)).sum()
    assert want > 0.0
    assert abs(t["br"] - want) < 1e-12 * want


def _dc_outage_flows(c, pbar, k):
    """Flows on every branch after branch k opens: a fresh solve of the
    reduced Laplacian (reference bus 0) of the network without k."""
    N, L = c.n_bus, c.n_branch
    y = c.br_x / (c.br_r ** 2 + c.br_x ** 2)
    keep = [l for l in range(L) if l != k]
    B = np.zeros((N, N))
    for l in keep:
        f, t = int(c.br_from[l]), int(c.br_to[l])
        B[f, f] += y[l]; B[t, t] += y[l]; B[f, t] -= y[l]; B[t, f] -= y[l]
    out = np.zeros((pbar.shape[0], L))
    for tt in range(pbar.shape[0]):
        th = np.zeros(N)
        th[1:] = np.linalg.solve(B[1:, 1:], pbar[tt, 1:])
        for l in keep:
            out[tt, l] = y[l] * (th[c.br_from[l]] - th[c.br_to[l]])
    return out


def test_contingency_term_from_complex_reactive_flows():
    """eqs. (sfr_pen)-(zctg) with the base-case reactive flows of the lossy AC
    model: z_tk = d_t c_s beta sum_{l != k} max(sqrt(P_tlk^2 + max(q_fr^2,
    q_to^2)_tl) - s_ctg_l, 0) at eps = 0, P from per-outage DC re-solves, q
    from complex power; the per-period max and mean over k."""
    c = _lossy_case(**MESH4, T=2, seed=41, ctg=[0, 1, 2, 3, 4])
    c.dt = np.array([1.0, 0.75])
    m = ob.make_model(c)
    T, N, G = c.n_period, c.n_bus, c.n_gen
    rng = np.random.default_rng(42)
    v, th, Vc = _phasors(rng, T, N)
    P = rng.uniform(0.0, 1.0, size=(T, G))
    S_fr, S_to = _branch_power(c, Vc)
    q2 = np.maximum(S_fr.imag ** 2, S_to.imag ** 2)
    pinj = P - c.load_p                      # one generator per bus, in bus order
    pbar = pinj - pinj.mean(axis=1, keepdims=True)
    K = c.n_ctg
    flows = [_dc_outage_flows(c, pbar, k) for k in range(K)]
    c.br_smax_ctg = 0.6 * np.sqrt(np.mean([f ** 2 for f in flows], axis=(0, 1)) + q2.mean(axis=0))
    beta = 0.9
    z = np.zeros((T, K))
    for k in range(K):
        s = np.sqrt(flows[k] ** 2 + q2)
        e = np.maximum(s - c.br_smax_ctg[None, :], 0.0)
        e[:, k] = 0.0
        z[:, k] = c.dt * c.c_s * beta * e.sum(axis=1)
    x = ob.pack(c, v, th, P, np.zeros((T, G)), np.zeros((T, G)), np.ones((T, G)))
    t, _ = ob.evaluate(m, x, 0.0, beta, 1.0, want_grad=False)
    assert z.max() > 0.0
    assert abs(t["ctg_max"] - z.max(axis=1).sum()) < 1e-10 * z.max()
    assert abs(t["ctg_mean"] - z.mean(axis=1).sum()) < 1e-10 * z.max()
    # the reactive part matters here: without it the term differs
    z0 = np.zeros((T, K))
    for k in range(K):
        e = np.maximum(np.abs(flows[k]) - c.br_smax_ctg[None, :], 0.0)
        e[:, k] = 0.0
        z0[:, k] = c.dt * c.c_s * beta * e.sum(axis=1)
    assert abs(z0.mean(axis=1).sum() - z.mean(axis=1).sum()) > 1e-3 * z.max()


@pytest.mark.parametrize("seed", [3, 4])
def test_angle_and_voltage_gradient_of_lossy_flows_matches_complex_derivative(seed):
    """The oracle's reverse pass through lossy, charged branches: the gradient
    of a weighted sum of all four flows, taken through C_bal at a point where
    every mismatch is far from zero (so the soft-abs is the absolute value up
    to O(eps^2)), equals central differences of the same sum formed from
    complex power.  Thermal and angle prices are zero and no contingency is
    listed, so C_bal is the only term that depends on v and theta."""
    c = _lossy_case(**MESH4, T=1, seed=seed, c_s=0.0, c_ang=0.0)
    m = ob.make_model(c)
    rng = np.random.default_rng(50 + seed)
    v, th, _ = _phasors(rng, 1, c.n_bus)
    # large loads keep every mismatch positive: C_bal = sum c (dp + dq) + O(eps^2)
    c.load_p = np.full((1, c.n_bus), 50.0)
    c.load_q = np.full((1, c.n_bus), 50.0)
    G = c.n_gen
    zeros = np.zeros((1, G))

    def bal_complex(vv, tt):
        S_fr, S_to = _branch_power(c, vv * np.exp(1j * tt))
        dp = c.load_p.copy(); dq = c.load_q.copy()
        np.add.at(dp, (slice(None), c.br_from), S_fr.real)
        np.add.at(dp, (slice(None), c.br_to), S_to.real)
        np.add.at(dq, (slice(None), c.br_from), S_fr.imag)
        np.add.at(dq, (slice(None), c.br_to), S_to.imag)
        return (c.c_p * dp + c.c_q * dq).sum()

    x = ob.pack(c, v, th, zeros, zeros, zeros, np.ones((1, G)))
    _, g = ob.evaluate(m, x, 1e-9, 1.0, 1.0)
    sl = c.block_slices()
    h = 1e-6
    for i in range(c.n_bus):
        for blk, arr in ((0, v), (1, th)):
            ap = arr.copy(); ap[0, i] += h
            am = arr.copy(); am[0, i] -= h
            if blk == 0:
                fd = (bal_complex(ap, th) - bal_complex(am, th)) / (2 * h)
            else:
                fd = (bal_complex(v, ap) - bal_complex(v, am)) / (2 * h)
            got = g[sl[blk]][i]
            assert abs(got - fd) < 1e-6 * max(1.0, abs(fd)), (blk, i, got, fd)
