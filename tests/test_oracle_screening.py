"""Pins of the oracle's contingency screening (Alg. 2) and of the screened
objective: the published SplitMix64 outputs, hand-derived selections,
brute-force contingency re-solves, finite differences and special cases that
reduce to the exact path."""
import json
import math
import os

import numpy as np
import pytest

from oracle import adam, objective as ob, screening as sc, solve
from paper_2310_06650_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MASK = (1 << 64) - 1


def _sequential(seed, n):
    """First n outputs of SplitMix64 run as a stream (state advanced by the
    increment once per output)."""
    out, state = [], seed
    for _ in range(n):
        state = (state + sc.GAMMA) & MASK
        out.append(sc.splitmix64_mix(state))
    return out


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64.json")) as f:
        gold = json.load(f)
    got = _sequential(gold["seed"], len(gold["outputs_hex"]))
    assert [f"{v:016x}" for v in got] == gold["outputs_hex"]


def test_key_is_the_counter_form_of_the_stream():
    """key(seed, 0, k) is output k + 1 of the stream: the closed-form counter
    and the running sum of increments agree."""
    for seed in (0, 12345, MASK - 7):
        assert [sc.key(seed, 0, k) for k in range(10)] == _sequential(seed, 10)


def test_counts():
    assert sc.counts(100, 0.1, 0.05) == (10, 15)
    assert sc.counts(7, 0.1, 0.1) == (1, 2)        # ceilings
    assert sc.counts(10, 0.8, 0.5) == (8, 10)      # capped at K
    assert sc.counts(10, 0.0, 0.0) == (0, 0)


def test_select_hand_example():
    """Eligible (sev > 0.5): 0 (3), 2 (5), 3 (5), 4 (1), 6 (2); by decreasing
    severity with the smaller index first on the tie: 2, 3, 0, 6, 4, so the
    worst three are {0, 2, 3}.  The two drawn from {1, 4, 5, 6} are the two
    smallest keys."""
    sev = np.array([3.0, 0.0, 5.0, 5.0, 1.0, 0.0, 2.0])
    seed, r = 99, 4
    got = sc.select(sev, 3, 5, 0.5, seed, r)
    rest = [1, 4, 5, 6]
    keys = {k: sc.key(seed, r, k) for k in rest}
    drawn = sorted(rest, key=lambda k: keys[k])[:2]
    assert list(got) == sorted([0, 2, 3] + drawn)


def test_select_threshold_leaves_worst_set_short():
    """Only two contingencies exceed zeta: the worst set holds those two and
    the draw fills the remaining slots."""
    sev = np.array([0.0, 9.0, 0.2, 4.0, 0.3, 0.0])
    got = sc.select(sev, 4, 5, 1.0, 7, 0)
    assert len(got) == 5 and {1, 3} <= set(got)
    assert len(set(got)) == 5 and list(got) == sorted(got)


def test_select_everything_and_nothing():
    sev = np.linspace(0.0, 1.0, 12)
    assert list(sc.select(sev, 3, 12, 0.0, 1, 2)) == list(range(12))
    assert list(sc.select(sev, 0, 0, 0.0, 1, 2)) == []
    # no worst slots: a pure draw
    got = sc.select(sev, 0, 4, 0.0, 1, 2)
    assert len(got) == 4


def test_select_worst_set_is_a_valid_top():
    rng = np.random.default_rng(3)
    sev = np.round(rng.exponential(1.0, 200), 1)        # many ties
    sev[rng.random(200) < 0.3] = 0.0
    zeta = 0.2
    got = set(sc.select(sev, 30, 50, zeta, 5, 1))
    order = sorted([k for k in range(200) if sev[k] > zeta], key=lambda k: (-sev[k], k))
    worst = order[:30]
    assert set(worst) <= got
    # every eligible contingency left out ranks after every one taken
    for k in order[30:]:
        for j in worst:
            assert (sev[j], -j) > (sev[k], -k)


def test_random_set_is_uniform():
    """With nothing eligible the set is a uniform draw of n_act of K: over
    2000 refreshes each contingency is taken 2000 n_act / K = 500 times, with
    a binomial spread of 19.4."""
    K, n_act, R = 40, 10, 2000
    sev = np.zeros(K)
    cnt = np.zeros(K)
    for r in range(R):
        got = sc.select(sev, 5, n_act, 0.0, 2024, r)
        assert len(got) == n_act
        cnt[got] += 1
    assert np.abs(cnt - R * n_act / K).max() < 5 * math.sqrt(R * 0.25 * 0.75)


# ---------------------------------------------------------------- screened objective

def _few_overloads_case():
    """c1 with the contingency ratings raised on all but two branches, so that
    only some outages overload anything."""
    c = synth.config_case("c1")
    c.br_smax_ctg = c.br_smax_ctg.copy()
    keep = np.zeros(c.n_branch, dtype=bool)
    keep[[3, 11]] = True
    c.br_smax_ctg[~keep] = 1e3
    return c


def test_excess_is_zero_without_overload_and_matches_bruteforce():
    c = _few_overloads_case()
    m = ob.make_model(c)
    x = synth.random_point(c, 2)
    eps, beta = 0.02, 0.9
    ex = ob.ctg_excess(m, x, eps, beta)
    _, _, zb = ob.ctg_term_bruteforce(m, x, eps, beta, return_z=True)
    floor = (c.dt * c.c_s * beta * (c.n_branch - 1) * eps)[:, None]
    assert np.abs(ex - (zb - floor)).max() <= 1e-10 * np.abs(zb).max()
    sev = sc.severity(m, x, eps, beta)
    assert (sev == 0.0).any() and (sev > 0.0).any()
    # a zero severity is exactly zero: no branch of that outage is overloaded
    for k in np.nonzero(sev == 0.0)[0]:
        assert np.all(zb[:, k] <= floor[:, 0] * (1 + 1e-12))


def test_screened_terms_match_bruteforce():
    """Scored contingencies take their re-solved penalty, the others the
    no-overload value; max and mean over all K."""
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 3)
    eps, beta = 0.02, 0.9
    active = np.array([1, 4, 5, 9, 13])
    t, _ = ob.evaluate(m, x, eps, beta, 1.0, want_grad=False, active=active)
    _, _, zb = ob.ctg_term_bruteforce(m, x, eps, beta, return_z=True)
    z = np.tile((c.dt * c.c_s * beta * (c.n_branch - 1) * eps)[:, None], (1, zb.shape[1]))
    z[:, active] = zb[:, active]
    assert abs(t["ctg_max"] - z.max(axis=1).sum()) <= 1e-10 * abs(t["ctg_max"])
    assert abs(t["ctg_mean"] - z.mean(axis=1).sum()) <= 1e-10 * abs(t["ctg_mean"])
    full, _ = ob.evaluate(m, x, eps, beta, 1.0, want_grad=False)
    assert t["ctg_mean"] < full["ctg_mean"]      # every left-out outage overloads here


def test_screened_gradient_matches_central_differences():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 4)
    eps, beta, rho = 0.05, 0.7, 0.8
    active = np.array([0, 2, 3, 8, 15])
    _, g = ob.evaluate(m, x, eps, beta, rho, active=active)
    _, gf = ob.evaluate(m, x, eps, beta, rho)
    rng = np.random.default_rng(11)
    sl = c.block_slices()
    p_slice = sl[2]
    assert np.abs(g[p_slice] - gf[p_slice]).max() > 1e-3 * np.abs(gf[p_slice]).max()
    for s in (sl[0], sl[1], sl[2], sl[3]):
        idx = rng.choice(np.arange(s.start, s.stop), size=12, replace=False)
        fd = []
        for j in idx:
            h = 1e-6 * max(1.0, abs(x[j]))
            xp = x.copy(); xp[j] += h
            xm = x.copy(); xm[j] -= h
            fp = ob.evaluate(m, xp, eps, beta, rho, want_grad=False, active=active)[0]
            fm = ob.evaluate(m, xm, eps, beta, rho, want_grad=False, active=active)[0]
            fd.append(sum(fp[k] - fm[k] for k in ob.TERMS if k != "load_value") / (2 * h))
        err = np.abs(np.array(fd) - g[idx]).max() / max(np.abs(g[s]).max(), 1e-30)
        assert err < 2e-7, (s, err)


def test_superset_of_overloaded_outages_is_exact():
    """Leaving out only outages without any overload changes nothing."""
    c = _few_overloads_case()
    m = ob.make_model(c)
    x = synth.random_point(c, 2)
    eps, beta = 0.02, 0.9
    sev = sc.severity(m, x, eps, beta)
    active = np.nonzero(sev > 0.0)[0]
    assert 0 < len(active) < len(sev)
    t, g = ob.evaluate(m, x, eps, beta, 1.0, active=active)
    tf, gf = ob.evaluate(m, x, eps, beta, 1.0)
    for k in ob.TERMS:
        assert abs(t[k] - tf[k]) <= 1e-12 * max(abs(tf[k]), 1.0), k
    assert np.abs(g - gf).max() <= 1e-12 * np.abs(gf).max()


def test_all_active_is_the_exact_objective():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x = synth.random_point(c, 6)
    t, g = ob.evaluate(m, x, 0.03, 1.0, 1.0, active=np.arange(len(m.ctg)))
    tf, gf = ob.evaluate(m, x, 0.03, 1.0, 1.0)
    assert t == tf and np.array_equal(g, gf)


# ---------------------------------------------------------------- screened loop

OPTS = dict(eps0=1e-2, epsf=1e-3, beta0=0.5, betaf=1.0, rho0=0.5, rhof=1.0,
            alpha0=[1e-3] * 6, alphaf=[1e-3] * 6, n_total=20)


def test_screened_loop_with_every_contingency_is_the_plain_loop():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x0 = synth.flat_start(c)
    scr = dict(top_frac=1.0, rand_frac=0.0, zeta=0.0, refresh=3, seed=1)
    x, mm, v, h, sets = sc.run(m, x0, 6, OPTS, scr)
    xr, mr, vr, hr = solve.run(m, x0, 6, OPTS)
    assert np.array_equal(x, xr) and np.array_equal(mm, mr) and h == hr


def test_screened_loop_refresh_points():
    c = synth.config_case("c1")
    m = ob.make_model(c)
    x0 = synth.flat_start(c)
    scr = dict(top_frac=0.25, rand_frac=0.125, zeta=0.0, refresh=3, seed=1)
    K = len(m.ctg)
    *_, sets = sc.run(m, x0, 7, OPTS, scr)
    assert [i for i, _ in sets] == [1, 4, 7]
    assert all(len(s) == sc.counts(K, 0.25, 0.125)[1] for _, s in sets)
    # a resumed run without a set refreshes at its first step
    *_, sets = sc.run(m, x0, 5, OPTS, scr, iter0=2)
    assert [i for i, _ in sets] == [3, 4, 7]
