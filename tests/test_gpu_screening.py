"""Contingency screening (Alg. 2) on the GPU against the FP64 oracle.

Screened evaluations (a given set) agree with the oracle's screened
objective to 1e-9 like the exact path; the device selection (severities,
worst set, SplitMix64 draw) reproduces the oracle's selection exactly, on
cases where the oracle's own severities leave the decisions well separated
(checked first, so a near tie fails loudly instead of flipping a set); the
screened Adam loop follows the oracle's screened loop.
"""
import numpy as np
import pytest

from oracle import objective as ob
from oracle import screening as osc
from paper_2310_06650_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-9
PREC = {"fp32": 1e-5, "bf16": 1e-3}


@pytest.fixture(scope="module")
def qg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_06650_amd import qg as _qg
    return _qg


_models = {}


def model(c):
    if id(c) not in _models:
        _models[id(c)] = ob.make_model(c)
    return _models[id(c)]


_cases = {}


def case(name):
    if name not in _cases:
        if name == "c2-sparse":
            # contingency ratings raised to 1.1 times the largest base-case
            # loading at the flat start: there, overloads come from outages
            # alone, and most outages overload nothing
            c = synth.config_case("c2")
            m0 = ob.make_model(c)
            V, TH, P, *_ = ob.unpack(c, synth.flat_start(c))
            q2, _ = ob.qmax2(ob.branch_flows(m0, V, TH))
            F = ob.balanced_injection(c, P) @ m0.isf.T
            c.br_smax_ctg = np.maximum(c.br_smax_ctg, 1.1 * np.sqrt(F * F + q2).max(axis=0))
        elif name == "c1-sparse":
            c = synth.config_case("c1")
            c.br_smax_ctg = c.br_smax_ctg.copy()
            keep = np.zeros(c.n_branch, dtype=bool)
            keep[[3, 11]] = True
            c.br_smax_ctg[~keep] = 1e3
        else:
            c = synth.config_case(name)
        c.name = name
        _cases[name] = c
    return _cases[name]


def close_terms(qg, got, ref, tol):
    got = dict(zip(qg.TERM_NAMES, got))
    scale = sum(abs(ref[k]) for k in ob.TERMS)
    for k in ob.TERMS + ("total",):
        assert abs(got[k] - ref[k]) <= tol * max(abs(ref[k]), 1e-12 * scale), (k, got[k], ref[k])


def close_grad(c, g, gr, tol):
    for name, s in zip(("v", "theta", "p", "q", "r", "u"), c.block_slices()):
        err = np.abs(g[s] - gr[s]).max() / max(np.abs(gr[s]).max(), 1e-300)
        assert err <= tol, (name, err)


def gpu_eval(prob, x, eps, beta, rho):
    import torch
    t, g = prob.eval_grad(prob.new_vector(x), eps, beta, rho)
    torch.cuda.synchronize()
    return t.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("name,n_act,seed,tile", [("c1", 5, 1, None), ("c2", 100, 2, None),
                                                  ("c2", 100, 2, "s4x2x3"), ("c2", 64, 3, None),
                                                  ("c2", 1, 4, "s2x3"), ("c2", 1, 4, None),
                                                  ("c3", 300, 5, None), ("c3", 300, 5, "8x8x7x4")])
def test_given_set_matches_oracle(qg, name, n_act, seed, tile):
    """Sets spanning several 64-slot chunks with a ragged tail, one slot, and
    the 2,410-contingency grid, under both tile forms."""
    c = case(name)
    prob = qg.Problem(c)
    if tile:
        prob.set_tile(tile)
    K = prob.K
    prob.set_screening(top_frac=n_act / K, rand_frac=0.0)
    rng = np.random.default_rng(seed)
    A = np.sort(rng.choice(K, size=n_act, replace=False))
    prob.set_active_contingencies(A)
    assert np.array_equal(prob.active_contingencies(), A)
    x = synth.random_point(c, seed, spread=0.3)
    t, g = gpu_eval(prob, x, 1e-2, 0.9, 1.0)
    tr, gr = ob.evaluate(model(c), x, 1e-2, 0.9, 1.0, active=A)
    close_terms(qg, t, tr, TOL)
    close_grad(c, g, gr, TOL)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_given_set_reduced_precision(qg, prec):
    c = case("c2")
    flags = qg.QG_FLAG_CTG_FP32 if prec == "fp32" else qg.QG_FLAG_CTG_BF16
    prob = qg.Problem(c, flags=flags)
    prob.set_tile("s4x2")
    prob.set_screening(top_frac=0.2, rand_frac=0.0)
    A = np.sort(np.random.default_rng(8).choice(prob.K, size=prob.K // 5, replace=False))
    prob.set_active_contingencies(A)
    x = synth.random_point(c, 8, spread=0.3)
    t, g = gpu_eval(prob, x, 1e-2, 1.0, 1.0)
    tr, gr = ob.evaluate(model(c), x, 1e-2, 1.0, 1.0, active=A)
    close_terms(qg, t, tr, PREC[prec])
    close_grad(c, g, gr, PREC[prec])


def test_every_contingency_in_the_set_is_the_exact_path(qg):
    """All K in the set: the same slots, factors and sums as the exact path,
    so the results are bitwise equal; turning screening off restores it."""
    c = case("c2")
    x = synth.random_point(c, 9, spread=0.3)
    ref = qg.Problem(c)
    t0, g0 = gpu_eval(ref, x, 1e-2, 1.0, 1.0)
    prob = qg.Problem(c)
    prob.set_screening(top_frac=1.0)
    prob.set_active_contingencies(np.arange(prob.K))
    t1, g1 = gpu_eval(prob, x, 1e-2, 1.0, 1.0)
    assert np.array_equal(t0, t1) and np.array_equal(g0, g1)
    prob.set_screening(None)
    t2, g2 = gpu_eval(prob, x, 1e-2, 1.0, 1.0)
    assert np.array_equal(t0, t2) and np.array_equal(g0, g2)


def _separated(sev, n_top, zeta, rel=1e-9):
    """The oracle's decisions are far from ties: no severity near zeta, and
    the last worst slot is clearly above the first one left out."""
    scale = max(sev.max(), 1e-300)
    nz = sev != 0.0   # exact zeros (no overload) are decided exactly on both sides
    assert np.all(np.abs(sev[nz] - zeta) > rel * scale)
    elig = np.sort(sev[sev > zeta])[::-1]
    if 0 < n_top < len(elig):
        assert elig[n_top - 1] - elig[n_top] > rel * scale


@pytest.mark.parametrize("name,top,rand,zeta_q,point", [
    ("c2-sparse", 0.1, 0.05, 0.0, "flat"),
    ("c2-sparse", 0.3, 0.1, 0.0, "flat"),      # fewer eligible than worst slots
    ("c2", 0.1, 0.1, 0.5, "random"),           # zeta at the median severity
    ("c2", 0.15, 0.0, 0.0, "flat"),
    ("c3", 0.05, 0.05, 0.0, "random")])
def test_refresh_selects_like_the_oracle(qg, name, top, rand, zeta_q, point):
    import torch
    c = case(name)
    m = model(c)
    prob = qg.Problem(c)
    x = synth.random_point(c, 12, spread=0.3) if point == "random" else synth.flat_start(c)
    eps, beta, rho = 1e-2, 0.8, 1.0
    sev_ref = osc.severity(m, x, eps, beta)
    zeta = float(np.quantile(sev_ref, zeta_q)) * (1 + 1e-6) if zeta_q else 0.0
    K = len(sev_ref)
    n_top, n_act = osc.counts(K, top, rand)
    _separated(sev_ref, n_top, zeta)
    prob.set_screening(top_frac=top, rand_frac=rand, zeta=zeta, refresh=5, seed=77)
    prob.screen_refresh(prob.new_vector(x), eps, beta, rho, round=3)
    ks, sev = prob.active_contingencies(severities=True)
    torch.cuda.synchronize()
    zero = sev_ref == 0.0
    assert np.array_equal(sev == 0.0, zero)
    assert np.abs(sev - sev_ref).max() <= TOL * sev_ref.max()
    want = osc.select(sev_ref, n_top, n_act, zeta, 77, 3)
    assert np.array_equal(ks, want)
    if name == "c2-sparse":
        assert zero.sum() > K // 4


def _solve_opts(qg, n, n_total=20, **kw):
    return qg.solve_opts(n, [1e-3] * 6, n_total=n_total, eps0=1e-2, epsf=1e-3, beta0=0.5,
                         betaf=1.0, rho0=0.5, rhof=1.0, **kw)


ORACLE_OPTS = dict(eps0=1e-2, epsf=1e-3, beta0=0.5, betaf=1.0, rho0=0.5, rhof=1.0,
                   alpha0=[1e-3] * 6, alphaf=[1e-3] * 6, n_total=20)


@pytest.mark.parametrize("name", ["c1-sparse", "c2-sparse"])
def test_screened_solve_follows_the_oracle(qg, name):
    """12 screened Adam steps, exact refreshes at steps 1 and 7 (refresh 6):
    one step per call without graphs, and one call of 12 steps replaying
    5-step graphs, give bitwise the same states; both follow the oracle's
    screened loop to 1e-9 and choose the same sets."""
    import torch
    c = case(name)
    m = model(c)
    scr = dict(top_frac=0.25, rand_frac=0.125, zeta=0.0, refresh=6, seed=5)
    x0 = synth.flat_start(c)
    rec = []
    osc.run(m, x0, 12, ORACLE_OPTS, scr, record=rec)
    prob = qg.Problem(c)
    prob.set_screening(scr["top_frac"], scr["rand_frac"], scr["zeta"], scr["refresh"],
                       scr["seed"])
    xd, md, vd = prob.new_vector(x0), prob.new_vector(), prob.new_vector()
    for i in range(12):
        prob.solve(xd, md, vd, _solve_opts(qg, 1, iter0=i, use_graph=0))
        torch.cuda.synchronize()
        xr, mr, _, ar = rec[i]
        xi = xd.cpu().numpy()
        assert np.abs(xi - xr).max() <= TOL * np.abs(xr).max(), ("x", i)
        assert np.array_equal(prob.active_contingencies(), ar), ("set", i)
    x_step = xd.cpu().numpy().copy()
    prob2 = qg.Problem(c)
    prob2.set_screening(scr["top_frac"], scr["rand_frac"], scr["zeta"], scr["refresh"],
                        scr["seed"])
    xg, mg, vg = prob2.new_vector(x0), prob2.new_vector(), prob2.new_vector()
    prob2.solve(xg, mg, vg, _solve_opts(qg, 12, use_graph=1))
    torch.cuda.synchronize()
    assert np.array_equal(xg.cpu().numpy(), x_step)


def test_screened_solve_reports_the_exact_score(qg):
    """The final score of a screened solve is evaluated with every
    contingency: it equals an exact evaluation at the returned point."""
    import torch
    c = case("c2")
    prob = qg.Problem(c)
    prob.set_screening(0.1, 0.05, 0.0, 8, 3)
    x0 = synth.flat_start(c)
    xd, md, vd = prob.new_vector(x0), prob.new_vector(), prob.new_vector()
    rep = prob.solve(xd, md, vd, _solve_opts(qg, 20, use_graph=1))
    assert rep.steps_done == 20
    torch.cuda.synchronize()
    ref = qg.Problem(c)
    t, _ = ref.eval_grad(xd, 0.0, 1.0, 1.0, grad=False)
    torch.cuda.synchronize()
    assert rep.final_score == -float(t.cpu().numpy()[qg.TERM_NAMES.index("total")])


def test_screening_argument_errors(qg):
    c = case("c1")
    prob = qg.Problem(c)
    K = prob.K
    with pytest.raises(qg.QgError):
        prob.screen_refresh(prob.new_vector(synth.flat_start(c)), 1e-2)   # screening off
    with pytest.raises(qg.QgError):
        prob.set_screening(top_frac=0.0, rand_frac=0.0)                   # empty set
    with pytest.raises(qg.QgError):
        prob.set_screening(top_frac=1.5)
    with pytest.raises(qg.QgError):
        prob.set_screening(top_frac=0.2, refresh=0)
    prob.set_screening(top_frac=0.25, rand_frac=0.0)
    cap = int(np.ceil(0.25 * K))
    with pytest.raises(qg.QgError):
        prob.set_active_contingencies(np.arange(cap + 1))                 # beyond the buffer
    with pytest.raises(qg.QgError):
        prob.set_active_contingencies([3, 1])                             # not increasing
    with pytest.raises(qg.QgError):
        prob.set_active_contingencies([0, K])                             # out of range
    x = prob.new_vector(synth.flat_start(c))
    m, v = prob.new_vector(), prob.new_vector()
    with pytest.raises(qg.QgError):
        prob.solve(x, m, v, _solve_opts(qg, 2, profile=1))
    with pytest.raises(qg.QgError):
        qg.solve_batch([prob], [x], [m], [v], _solve_opts(qg, 2))


def test_refresh_cycles_across_schedule_chunks(qg):
    """Refresh every 7 steps while the schedule is uploaded in chunks of 10
    (check_every): whole cycles replay as graphs, cycles cut by a chunk end
    run as plain launches; states and sets equal a solve without graphs
    bitwise."""
    import torch
    c = case("c2-sparse")
    outs = []
    for use_graph in (0, 1):
        prob = qg.Problem(c)
        prob.set_screening(0.1, 0.05, 0.0, 7, 11)
        x0 = synth.flat_start(c)
        xd, md, vd = prob.new_vector(x0), prob.new_vector(), prob.new_vector()
        prob.solve(xd, md, vd, _solve_opts(qg, 30, n_total=30, check_every=10,
                                           use_graph=use_graph))
        torch.cuda.synchronize()
        outs.append((xd.cpu().numpy(), md.cpu().numpy(), prob.active_contingencies()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])
