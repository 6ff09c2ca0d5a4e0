"""Warm-start network kernels (FP32 MFMA training, BF16 inference) against the
FP64 NumPy oracle of the same network.

Tolerances: FP32 products of length K carry a relative error of about
sqrt(K) 2^-24 per output (K <= 700 here: < 2e-6), and the reverse pass
chains three such layers, so outputs, loss and gradients are compared at
2e-5 normwise per array.  BF16 operands carry 2^-9 relative rounding per
weight and activation; the BF16 forward is compared at 3e-2 normwise.
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_06650_amd import qg as _qg
    return _qg


def make(qg, d_in, width, depth, d_out, batch, seed):
    import torch
    net = qg.MLP(d_in, width, depth, d_out, max_batch=batch)
    rng = np.random.default_rng(seed)
    sizes = [d_in] + [width] * depth + [d_out]
    params = []
    flat = np.zeros(net.n_params, dtype=np.float32)
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        W = rng.normal(0, 1.0 / np.sqrt(a), (a, b)).astype(np.float32)
        bb = rng.normal(0, 0.1, b).astype(np.float32)
        wo, bo = net.offsets(i)
        flat[wo:wo + a * b] = W.reshape(-1)
        flat[bo:bo + b] = bb
        params.append((W.astype(np.float64), bb.astype(np.float64)))
    net.set_params(flat)
    x = rng.normal(size=(batch, d_in)).astype(np.float32)
    t = rng.normal(size=(batch, d_out)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    return net, params, x.astype(np.float64), t.astype(np.float64), xd, td


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


SHAPES = [(37, 48, 3, 53, 19), (700, 64, 2, 600, 5), (11, 130, 1, 7, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_loss_and_gradient(qg, shape):
    import torch
    net, params, x, t, xd, td = make(qg, *shape, seed=sum(shape))
    y = net.forward(xd)
    torch.cuda.synchronize()
    y_ref = omlp.forward(params, x)
    assert rel(y.cpu().numpy(), y_ref) < 2e-5
    g, loss = net.grad_and_loss(xd, td)
    torch.cuda.synchronize()
    loss_ref, grads_ref = omlp.loss_and_grad(params, x, t)
    assert abs(float(loss) - loss_ref) <= 2e-5 * loss_ref
    g = g.cpu().numpy()
    for i, (dW, db) in enumerate(grads_ref):
        wo, bo = net.offsets(i)
        assert rel(g[wo:wo + dW.size].reshape(dW.shape), dW) < 2e-5, ("W", i)
        assert rel(g[bo:bo + db.size], db) < 2e-5, ("b", i)


# the network of the learned warm start: 617-bus x 18-period loads and
# reserves in, 3 x 512 GELU, every variable of the grid out, batch 64
C5_SHAPE = (11124, 512, 3, 29412, 64)


def test_forward_loss_and_gradient_c5_shape(qg):
    """The real warm-start network.  Products of up to 11,124 FP32 terms carry
    about sqrt(11124) 2^-24 = 6e-6 relative error per output, and the reverse
    pass chains four layers: outputs, loss and every gradient array are
    compared at 1e-4 normwise; the BF16 forward at 3e-2."""
    import torch
    net, params, x, t, xd, td = make(qg, *C5_SHAPE, seed=11)
    y = net.forward(xd)
    torch.cuda.synchronize()
    y_ref = omlp.forward(params, x)
    assert rel(y.cpu().numpy(), y_ref) < 1e-4
    g, loss = net.grad_and_loss(xd, td)
    torch.cuda.synchronize()
    loss_ref, grads_ref = omlp.loss_and_grad(params, x, t)
    assert abs(float(loss) - loss_ref) <= 1e-4 * loss_ref
    g = g.cpu().numpy()
    for i, (dW, db) in enumerate(grads_ref):
        wo, bo = net.offsets(i)
        assert rel(g[wo:wo + dW.size].reshape(dW.shape), dW) < 1e-4, ("W", i)
        assert rel(g[bo:bo + db.size], db) < 1e-4, ("b", i)
    y16 = net.forward_bf16(xd)
    torch.cuda.synchronize()
    assert rel(y16.cpu().numpy(), y_ref) < 3e-2


def test_train_step_is_grad_then_adam(qg):
    import torch
    net, params, x, t, xd, td = make(qg, 37, 48, 3, 53, 19, seed=5)
    p0 = net.params.cpu().numpy().astype(np.float64)
    net.train_step(xd, td, 1e-3)
    torch.cuda.synchronize()
    p1 = net.params.cpu().numpy().astype(np.float64)
    _, grads_ref = omlp.loss_and_grad(params, x, t)
    for i, (dW, db) in enumerate(grads_ref):
        wo, bo = net.offsets(i)
        for off, g in ((wo, dW.reshape(-1)), (bo, db)):
            sl = slice(off, off + g.size)
            want, _, _ = omlp.adam(p0[sl], np.zeros(g.size), np.zeros(g.size), g, 1, 1e-3)
            # the first Adam step moves each entry by about lr sign(g): compare
            # the steps, where FP32 gradients of near-zero entries may flip sign
            step, step_ref = p1[sl] - p0[sl], want - p0[sl]
            big = np.abs(g) > 1e-3 * np.abs(g).max()
            assert np.allclose(step[big], step_ref[big], rtol=1e-4, atol=1e-9)


def test_training_reduces_the_loss(qg):
    import torch
    net, params, x, t, xd, td = make(qg, 37, 48, 3, 53, 19, seed=6)
    first = float(net.train_step(xd, td, 3e-3))
    for _ in range(200):
        last = net.train_step(xd, td, 3e-3)
    torch.cuda.synchronize()
    assert float(last) < 0.2 * first


@pytest.mark.parametrize("shape", SHAPES)
def test_bf16_forward(qg, shape):
    import torch
    net, params, x, t, xd, td = make(qg, *shape, seed=7 + sum(shape))
    y32 = net.forward(xd).cpu().numpy()
    y16 = net.forward_bf16(xd)
    torch.cuda.synchronize()
    assert rel(y16.cpu().numpy(), omlp.forward(params, x)) < 3e-2
    assert rel(y16.cpu().numpy(), y32) < 3e-2


def test_deterministic(qg):
    import torch
    net, params, x, t, xd, td = make(qg, 700, 64, 2, 600, 5, seed=9)
    a = net.forward(xd).cpu().numpy()
    g1 = net.grad_and_loss(xd, td)[0].cpu().numpy().copy()
    b = net.forward(xd).cpu().numpy()
    g2 = net.grad_and_loss(xd, td)[0].cpu().numpy().copy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b) and np.array_equal(g1, g2)
