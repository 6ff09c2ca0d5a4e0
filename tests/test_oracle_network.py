"""Pins of the oracle's DC network algebra (Section II-E) against closed forms,
Kirchhoff's law and the brute-force per-outage re-solve."""
import json
import os

import numpy as np
import pytest

from oracle import network
from paper_2310_06650_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_three_bus_closed_form_flows():
    g = _gold("three_bus.json")
    E = network.incidence(g["n_bus"], np.array(g["br_from"]), np.array(g["br_to"]))
    y = np.array(g["susceptance"])
    p = np.array(g["p_bar"])
    f_solve = network.dc_flows_solve(E, y, p)
    f_isf = network.isf_matrix(E, y) @ p
    np.testing.assert_allclose(f_solve, g["flows"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(f_isf, g["flows"], rtol=0, atol=1e-15)


def test_three_bus_outage_and_lodf():
    g = _gold("three_bus.json")
    fr, to = np.array(g["br_from"]), np.array(g["br_to"])
    E = network.incidence(g["n_bus"], fr, to)
    y = np.array(g["susceptance"])
    p = np.array(g["p_bar"])
    k = g["outage"]["branch"]
    f_out = network.outage_flows(E, y, p, k)
    np.testing.assert_allclose(f_out, g["outage"]["flows"], atol=1e-15)
    isf = network.isf_matrix(E, y)
    lodf = network.lodf_matrix(isf, fr, to, np.array([k]))
    np.testing.assert_allclose(lodf[:, 0], g["outage"]["lodf_column"], atol=1e-14)


def test_susceptance_definition():
    # y = -b^sr with b^sr = -x/(r^2+x^2): pure reactance gives 1/x
    assert network.susceptance(np.array([0.0]), np.array([0.25]))[0] == 4.0
    y = network.susceptance(np.array([0.1]), np.array([0.2]))[0]
    assert abs(y - 0.2 / 0.05) < 1e-14


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_kirchhoff_and_ref_invariance(name):
    c = synth.config_case(name)
    E = network.incidence(c.n_bus, c.br_from, c.br_to)
    y = network.susceptance(c.br_r, c.br_x)
    rng = np.random.default_rng(3)
    p = rng.normal(size=(4, c.n_bus))
    p -= p.mean(axis=1, keepdims=True)
    isf0 = network.isf_matrix(E, y, ref=0)
    F = p @ isf0.T
    # nodal balance E^T f = p (Section II-E, injections = E^T (f + b), b = 0)
    np.testing.assert_allclose(F @ E, p, atol=1e-11 * np.abs(p).max())
    # a different reference bus gives the same flows for balanced injections
    isf5 = network.isf_matrix(E, y, ref=5)
    np.testing.assert_allclose(p @ isf5.T, F, atol=1e-11 * np.abs(F).max())
    # and so does the direct reduced solve
    np.testing.assert_allclose(network.dc_flows_solve(E, y, p), F,
                               atol=1e-11 * np.abs(F).max())
    # a uniform shift of injections is absorbed by the uniform slack only when
    # removed first: ISF @ 1 is not zero, ISF @ (1 - mean) is
    ones = np.ones(c.n_bus)
    np.testing.assert_allclose(isf0 @ (ones - ones.mean()), 0.0, atol=1e-13)


def test_bridges_match_generator_lists():
    c = synth.config_case("c1")
    br = network.bridges_bruteforce(c.n_bus, c.br_from, c.br_to)
    assert set(np.flatnonzero(~br)) == set(c.ctg_list.tolist())
    c2 = synth.config_case("c2")
    br2 = network.bridges_bruteforce(c2.n_bus, c2.br_from, c2.br_to)
    assert not br2[c2.ctg_list].any()
    assert c2.n_ctg == 560


@pytest.mark.parametrize("name,sample", [("c1", None), ("c2", 25)])
def test_lodf_equals_outage_resolve(name, sample):
    c = synth.config_case(name)
    E = network.incidence(c.n_bus, c.br_from, c.br_to)
    y = network.susceptance(c.br_r, c.br_x)
    isf = network.isf_matrix(E, y)
    ctg = np.asarray(c.ctg_list)
    lodf = network.lodf_matrix(isf, c.br_from, c.br_to, ctg)
    rng = np.random.default_rng(11)
    p = rng.normal(size=(3, c.n_bus))
    p -= p.mean(axis=1, keepdims=True)
    F = p @ isf.T
    ks = range(len(ctg)) if sample is None else rng.choice(len(ctg), sample, replace=False)
    for ki in ks:
        k = int(ctg[ki])
        f_ref = network.outage_flows(E, y, p, k)
        f_lodf = F + lodf[:, ki][None, :] * F[:, k][:, None]
        scale = np.abs(f_ref).max()
        np.testing.assert_allclose(f_lodf, f_ref, atol=1e-11 * scale)
        assert lodf[k, ki] == -1.0
        # post-outage conservation with the branch removed
        m = np.ones(c.n_branch, dtype=bool)
        m[k] = False
        np.testing.assert_allclose(f_lodf[:, m] @ E[m], p, atol=1e-10 * np.abs(p).max())


def test_sherman_morrison_angle_form_matches_resolve():
    """eq. (rank_correct): theta_k = theta_b - u_k (w_k^T c) equals the solve
    of the outaged system, for a rank-1 change sigma a a^T with sigma = -y_k."""
    c = synth.config_case("c1")
    E = network.incidence(c.n_bus, c.br_from, c.br_to)
    y = network.susceptance(c.br_r, c.br_x)
    keep = np.arange(c.n_bus) != 0
    Eh = E[:, keep]
    Y = Eh.T @ (y[:, None] * Eh)
    rng = np.random.default_rng(5)
    cvec = rng.normal(size=c.n_bus - 1)
    th_b = np.linalg.solve(Y, cvec)
    for k in c.ctg_list:
        a = Eh[k]
        sig = -y[k]
        u = np.linalg.solve(Y, a)
        w = sig * u / (1.0 + sig * a @ u)
        th_k = th_b - u * (w @ cvec)
        th_ref = np.linalg.solve(Y + sig * np.outer(a, a), cvec)
        np.testing.assert_allclose(th_k, th_ref, atol=1e-11 * np.abs(th_ref).max())
