"""The copper-plate yardstick z_ed: a closed-form case, and the bound
score(x) <= z_ed for points of the box (the property the gap ratio of
Section III relies on)."""
import numpy as np
import pytest

from _cases import tiny_case
from oracle import adam as oadam
from oracle import objective as ob
from oracle import solve as osolve
from paper_2310_06650_amd import ed, synth


def score(model, x, rho_scale=1.0):
    terms, _ = ob.evaluate(model, x, 0.0, 1.0, rho_scale, want_grad=False)
    return -terms["total"]


def test_closed_form_single_period():
    # 2 buses, 1 generator, 1 period: serve 0.4 pu from the first block
    # (10 $/pu h), carry the 0.1 pu reserve at 1 $/pu h; with c_on = c_sd = 1
    # the status costs 1 whatever u in [1/3, 1].  z = 60 * 0.4 - 5.1.
    c = tiny_case(2, [0], [1], [0.1], [0], T=1)
    r = ed.copper_plate(c)
    assert r.z_ed == pytest.approx(24.0 - 5.1, rel=1e-9)
    assert r.p[0, 0] == pytest.approx(0.4, rel=1e-9)
    assert r.r[0, 0] == pytest.approx(0.1, rel=1e-9)


def test_shortfall_cheaper_than_reserve():
    # reserve capability priced above the shortfall: the relaxation buys the
    # shortfall (c_rsv = 20 per pu h) instead of r at 30 per pu h
    c = tiny_case(2, [0], [1], [0.1], [0], T=1, gen_c_r=np.array([30.0]))
    r = ed.copper_plate(c)
    assert r.r[0, 0] == pytest.approx(0.0, abs=1e-12)
    assert r.z_ed == pytest.approx(24.0 - (4.0 + 1.0 + 20.0 * 0.1), rel=1e-9)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_bound_on_random_points(name):
    c = synth.config_case(name)
    z = ed.copper_plate(c).z_ed
    m = ob.make_model(c)
    for seed in range(6):
        x = synth.random_point(c, 100 + seed)
        assert score(m, x) <= z + 1e-9 * abs(z)
    assert score(m, synth.flat_start(c)) <= z + 1e-9 * abs(z)


def test_bound_along_an_adam_run():
    c = synth.config_case("c1")
    z = ed.copper_plate(c).z_ed
    m = ob.make_model(c)
    opts = dict(alpha0=[1e-3] * 6, alphaf=[1e-4] * 6, eps0=1e-1, epsf=1e-4, beta0=0.1,
                betaf=1.0, rho0=0.1, rhof=1.0)
    x = synth.flat_start(c)
    lo, hi = oadam.box_bounds(c)
    mm = np.zeros_like(x)
    vv = np.zeros_like(x)
    n = 60
    for i in range(1, n + 1):
        eps, beta, rho, alpha = osolve.schedule(i, n, opts)
        _, g = ob.evaluate(m, x, eps, beta, rho)
        x, mm, vv = oadam.adam_update(x, mm, vv, g, i, osolve.class_vector(c, alpha), lo, hi)
        assert score(m, x) <= z + 1e-9 * abs(z)
