"""qg_eval_grad_noalloc (static device scratch, no workspace argument)
against qg_eval_grad (caller's workspace) through the C ABI: two calls in a
row on one GPU, the second on a smaller problem, so the second runs on the
scratch the first left behind; and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2310_06650_amd import qg, synth
    return torch, qg, synth


def _both(torch, qg, prob, x, eps, beta, rho):
    t_ref, g_ref = prob.eval_grad(x, eps, beta, rho)
    g = torch.full((prob.n_x,), float("nan"), dtype=torch.float64, device=prob.device)
    t = torch.full((32,), float("nan"), dtype=torch.float64, device=prob.device)
    prob.eval_grad_noalloc(x, eps, beta, rho, grad=g, terms=t)
    torch.cuda.synchronize()
    return (t_ref.cpu().numpy(), g_ref.cpu().numpy(),
            t[:qg.QG_NTERMS].cpu().numpy(), g.cpu().numpy())


def test_noalloc_matches_workspace_entry_point_large_then_small():
    torch, qg, synth = _env()
    from oracle import objective as ob
    # first call: the 617-bus, 18-period benchmark grid (15 MB of scratch)
    big = synth.config_case("c2")
    pb = qg.Problem(big, device="cuda:0")
    assert pb.sizes.workspace_bytes <= qg.QG_NOALLOC_SCRATCH
    xb = pb.new_vector(synth.random_point(big, 7))
    print("noalloc: c2 617-bus call", flush=True)
    tr, gr, tn, gn = _both(torch, qg, pb, xb, 2e-2, 0.8, 0.6)
    assert np.isfinite(gn).all() and np.isfinite(tn).all()
    # the same kernels in the same order: the results are identical
    assert np.array_equal(tn, tr)
    assert np.array_equal(gn, gr)
    # second call, smaller: the 14-bus grid on the scratch the first left
    small = synth.config_case("c1")
    ps = qg.Problem(small, device="cuda:0")
    xs_h = synth.random_point(small, 8)
    xs = ps.new_vector(xs_h)
    print("noalloc: c1 14-bus call", flush=True)
    tr, gr, tn, gn = _both(torch, qg, ps, xs, 1e-2, 1.0, 1.0)
    assert np.array_equal(tn, tr)
    assert np.array_equal(gn, gr)
    # and against the FP64 oracle at the parity bar (1e-9 relative)
    to, go = ob.evaluate(ob.make_model(small), xs_h, 1e-2, 1.0, 1.0)
    tot = tn[qg.TERM_NAMES.index("total")]
    assert abs(tot - to["total"]) <= 1e-9 * abs(to["total"])
    for s in small.block_slices():
        assert np.abs(gn[s] - go[s]).max() <= 1e-9 * np.abs(go[s]).max()
    # terms only (no gradient output)
    t = torch.zeros(32, dtype=torch.float64, device="cuda:0")
    ps.eval_grad_noalloc(xs, 1e-2, 1.0, 1.0, grad=None, terms=t)
    torch.cuda.synchronize()
    assert np.array_equal(t[:qg.QG_NTERMS].cpu().numpy(), tr)
    pb.close()
    ps.close()


def test_noalloc_rejects_a_workspace_above_the_limit():
    torch, qg, synth = _env()
    case = synth.make_case(seed=5, n_bus=617, n_branch=850, n_gen=100, n_period=48)
    prob = qg.Problem(case, device="cuda:0")
    assert prob.sizes.workspace_bytes > qg.QG_NOALLOC_SCRATCH
    x = prob.new_vector(synth.flat_start(case))
    t = torch.zeros(32, dtype=torch.float64, device="cuda:0")
    with pytest.raises(qg.QgError) as ei:
        prob.eval_grad_noalloc(x, 1e-2, grad=None, terms=t)
    assert ei.value.status == qg.QG_ERR_ARG
    assert "exceeds the static scratch" in str(ei.value)
    prob.close()
