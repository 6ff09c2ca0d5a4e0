"""The C-ABI library loads, exports every symbol qg.h declares, and its
host-only entry point (qg_problem_sizes) validates inputs.  No GPU needed."""
import os
import re

import numpy as np
import pytest

from oracle import network
from paper_2310_06650_amd import synth
from tests._cases import tiny_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

qg = pytest.importorskip("paper_2310_06650_amd.qg",
                         reason="libqg.so not built (run __graft_entry__.build())")


def _declared_symbols():
    text = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                text += f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qg_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(qg.lib, n), n
        assert n in qg.EXPORTED, n


def test_status_strings():
    assert qg.lib.qg_status_string(0) == b"ok"
    assert b"topology" in qg.lib.qg_status_string(qg.QG_ERR_TOPOLOGY)


def _sizes(case, mode=None, ctg=None, **kw):
    desc, k1 = qg.grid_desc(case)
    if mode is None:
        mode = qg.QG_CTG_LIST
    opts, k2 = qg.build_opts(case, ctg_mode=mode, ctg_list=ctg, **kw)
    return qg.qg_problem_sizes(desc, opts)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_sizes_and_contingency_count(name):
    c = synth.config_case(name)
    s = _sizes(c)
    assert s.n_x == c.n_x and s.n_ctg == c.n_ctg
    assert s.const_bytes > 0 and s.workspace_bytes > 0
    s_all = _sizes(c, mode=qg.QG_CTG_ALL_NONBRIDGE)
    br = network.bridges_bruteforce(c.n_bus, c.br_from, c.br_to) if name == "c1" else None
    if br is not None:
        assert s_all.n_ctg == int((~br).sum())


def test_tree_grid_has_no_contingencies():
    c = tiny_case(4, [0, 1, 2], [1, 2, 3], [0.1, 0.1, 0.1], [0])
    s = _sizes(c, mode=qg.QG_CTG_ALL_NONBRIDGE)
    assert s.n_ctg == 0


def _expect(status, fn):
    with pytest.raises(qg.QgError) as e:
        fn()
    assert e.value.status == status, str(e.value)


def test_disconnected_grid_is_topology_error():
    c = tiny_case(4, [0, 2], [1, 3], [0.1, 0.1], [0])
    _expect(qg.QG_ERR_TOPOLOGY, lambda: _sizes(c, mode=qg.QG_CTG_ALL_NONBRIDGE))


def test_listed_bridge_is_topology_error():
    c = tiny_case(4, [0, 1, 2, 0], [1, 2, 3, 2], [0.1] * 4, [0])
    # branch 2 (2-3) is a bridge
    _expect(qg.QG_ERR_TOPOLOGY, lambda: _sizes(c, ctg=[0, 2]))
    assert _sizes(c, ctg=[0, 1, 3]).n_ctg == 3


def test_bad_values_are_arg_errors():
    c = tiny_case(3, [0, 1, 0], [1, 2, 2], [0.1, 0.1, 0.1], [0])
    bad = tiny_case(3, [0, 1, 0], [1, 2, 2], [0.1, -0.1, 0.1], [0])
    _expect(qg.QG_ERR_ARG, lambda: _sizes(bad, ctg=[]))
    oob = tiny_case(3, [0, 1, 0], [1, 5, 2], [0.1, 0.1, 0.1], [0])
    _expect(qg.QG_ERR_ARG, lambda: _sizes(oob, ctg=[]))
    loop = tiny_case(3, [0, 1, 0], [1, 1, 2], [0.1, 0.1, 0.1], [0])
    _expect(qg.QG_ERR_ARG, lambda: _sizes(loop, ctg=[]))
    _expect(qg.QG_ERR_ARG, lambda: _sizes(c, ctg=[0, 0]))
    _expect(qg.QG_ERR_ARG, lambda: _sizes(c, ctg=[7]))
    _expect(qg.QG_ERR_ARG, lambda: _sizes(c, ctg=[], ref_bus=9))
    c.gen_pmin = c.gen_pmax * 2
    _expect(qg.QG_ERR_ARG, lambda: _sizes(c, ctg=[]))
    long_t = tiny_case(3, [0, 1, 0], [1, 2, 2], [0.1, 0.1, 0.1], [0], T=65)
    _expect(qg.QG_ERR_ARG, lambda: _sizes(long_t, ctg=[]))


def test_parallel_branches_are_not_bridges():
    c = tiny_case(3, [0, 0, 1], [1, 1, 2], [0.1, 0.2, 0.1], [0])
    s = _sizes(c, mode=qg.QG_CTG_ALL_NONBRIDGE)
    assert s.n_ctg == 2   # the two parallel 0-1 branches; 1-2 is a bridge


def test_null_arguments():
    _expect(qg.QG_ERR_ARG, lambda: qg.qg_problem_sizes(qg.qg_grid_desc(), qg.qg_build_opts()))


def test_precision_flags_size_the_factor_storage():
    c = synth.config_case("c2")
    lp = (c.n_branch + 63) // 64 * 64
    kp = (c.n_ctg + 63) // 64 * 64
    s64 = _sizes(c).const_bytes
    s32 = _sizes(c, flags=qg.QG_FLAG_CTG_FP32).const_bytes
    s16 = _sizes(c, flags=qg.QG_FLAG_CTG_BF16).const_bytes
    # the factor array shrinks from 8 to 4 to 2 bytes per entry (256-B aligned)
    assert abs((s64 - s32) - 4 * lp * kp) <= 256
    assert abs((s32 - s16) - 2 * lp * kp) <= 256
    with pytest.raises(qg.QgError) as e:
        _sizes(c, flags=qg.QG_FLAG_CTG_FP32 | qg.QG_FLAG_CTG_BF16)
    assert e.value.status == qg.QG_ERR_ARG
    with pytest.raises(qg.QgError):
        _sizes(c, flags=0x100)


def test_load_draws_keep_the_grid():
    c = synth.config_case("c2")
    a = synth.load_draw(c, 10000)
    b = synth.load_draw(c, 10000)
    d = synth.load_draw(c, 10001)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    assert not np.array_equal(a[0], d[0])
    lp, lq, rr = a
    assert lp.shape == c.load_p.shape and (lp > 0).all()
    peak = lp.sum(axis=1).max() / c.load_p.sum(axis=1).max()
    assert 0.85 - 1e-12 <= peak <= 1.0 + 1e-12
    assert np.allclose(rr, 0.1 * lp.sum(axis=1))
    c2 = synth.with_loads(c, a)
    assert c2.n_bus == c.n_bus and np.array_equal(c2.br_x, c.br_x)


def test_sum_flag_and_period_limit():
    c = synth.config_case("c1")
    base = _sizes(c)
    s = _sizes(c, flags=qg.QG_FLAG_CTG_SUM | qg.QG_FLAG_CTG_FP32)
    assert s.n_x == base.n_x and s.workspace_bytes == base.workspace_bytes
    c65 = synth.config_case("c1")
    c65.n_period = 65
    T = 65
    c65.load_p = np.tile(c.load_p[:1], (T, 1))
    c65.load_q = np.tile(c.load_q[:1], (T, 1))
    c65.reserve_req = np.full(T, c.reserve_req[0])
    c65.dt = np.ones(T)
    with pytest.raises(qg.QgError) as e:
        _sizes(c65)
    assert e.value.status == qg.QG_ERR_ARG


def _image(case, mode=None, ctg=None):
    desc, k1 = qg.grid_desc(case)
    opts, k2 = qg.build_opts(case, ctg_mode=qg.QG_CTG_LIST if mode is None else mode,
                             ctg_list=ctg)
    sizes = qg.qg_problem_sizes(desc, opts)
    return qg.qg_build_image(desc, opts, sizes.const_bytes), sizes


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_host_build_image_is_deterministic(name):
    """The host part of the build (bridges, factor, shift and outage factors)
    fills the arena image the same way twice, to the last byte."""
    c = synth.config_case(name)
    a, sizes = _image(c)
    b, _ = _image(c)
    assert a.size == sizes.const_bytes
    assert np.array_equal(a, b)
    assert np.count_nonzero(a) > a.size // 10


def test_host_build_image_errors():
    c = synth.config_case("c1")
    desc, k1 = qg.grid_desc(c)
    opts, k2 = qg.build_opts(c)
    sizes = qg.qg_problem_sizes(desc, opts)
    with pytest.raises(qg.QgError) as ei:
        qg.qg_build_image(desc, opts, sizes.const_bytes - 1)
    assert ei.value.status == qg.QG_ERR_ARG
    # an outage that islands (a radial branch) in the list
    radial = tiny_case(4, [0, 1, 2, 0], [1, 2, 0, 3], [0.1, 0.2, 0.1, 0.1], [0, 1])
    with pytest.raises(qg.QgError) as ei:
        _image(radial, ctg=[3])
    assert ei.value.status == qg.QG_ERR_TOPOLOGY
    # a disconnected grid
    split = tiny_case(4, [0, 2], [1, 3], [0.1, 0.1], [0, 2])
    with pytest.raises(qg.QgError) as ei:
        _image(split)
    assert ei.value.status == qg.QG_ERR_TOPOLOGY
