"""Pins of the MLP oracle: GELU special values and its odd-part identity,
closed forms of degenerate networks, and finite differences."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_special_values():
    assert mlp.gelu(0.0) == 0.0
    assert mlp.gelu_grad(0.0) == pytest.approx(0.5, abs=1e-15)
    # gelu(z) - gelu(-z) = z (Phi(z) + Phi(-z) = 1)
    z = np.linspace(-6, 6, 97)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    # tails: z Phi(z) -> z for large z, -> 0 for very negative z
    assert mlp.gelu(12.0) == pytest.approx(12.0, rel=1e-15)
    assert abs(mlp.gelu(-12.0)) < 1e-30
    # Phi(1) from the error function's series at 1/sqrt(2)
    assert mlp.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)


def test_gelu_grad_finite_difference():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-9)


def _params(rng, sizes, scale=0.5):
    return [(rng.normal(0, scale, (a, b)), rng.normal(0, scale, b))
            for a, b in zip(sizes[:-1], sizes[1:])]


def test_zero_weights_give_the_bias_and_its_gradient():
    rng = np.random.default_rng(0)
    sizes = [5, 4, 4, 3]
    params = [(np.zeros((a, b)), np.zeros(b)) for a, b in zip(sizes[:-1], sizes[1:])]
    b_out = np.array([0.5, -1.0, 2.0])
    params[-1] = (np.zeros((4, 3)), b_out)
    x = rng.normal(size=(7, 5))
    t = rng.normal(size=(7, 3))
    y = mlp.forward(params, x)
    assert np.array_equal(y, np.tile(b_out, (7, 1)))
    loss, grads = mlp.loss_and_grad(params, x, t)
    assert loss == pytest.approx(((b_out - t) ** 2).mean(), rel=1e-14)
    assert np.allclose(grads[-1][1], 2 * (b_out - t).sum(axis=0) / t.size, atol=1e-15)
    # hidden activations are gelu(0) = 0, so every weight gradient vanishes
    for dW, _ in grads:
        assert np.all(dW == 0.0)


def test_one_unit_network_closed_form():
    # x -> gelu(w1 x + b1) -> w2 h + b2, one sample
    w1, b1, w2, b2, x, t = 0.7, -0.2, 1.3, 0.1, 0.9, 0.4
    params = [(np.array([[w1]]), np.array([b1])), (np.array([[w2]]), np.array([b2]))]
    z = w1 * x + b1
    phi_z = 0.5 * (1 + math.erf(z / math.sqrt(2)))
    h = z * phi_z
    y = w2 * h + b2
    loss, grads = mlp.loss_and_grad(params, np.array([[x]]), np.array([[t]]))
    assert loss == pytest.approx((y - t) ** 2, rel=1e-14)
    dy = 2 * (y - t)
    dz = dy * w2 * (phi_z + z * math.exp(-z * z / 2) / math.sqrt(2 * math.pi))
    assert grads[1][0][0, 0] == pytest.approx(dy * h, rel=1e-13)
    assert grads[1][1][0] == pytest.approx(dy, rel=1e-13)
    assert grads[0][0][0, 0] == pytest.approx(dz * x, rel=1e-13)
    assert grads[0][1][0] == pytest.approx(dz, rel=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    sizes = [6, 5, 4, 3]
    params = _params(rng, sizes)
    x = rng.normal(size=(4, 6))
    t = rng.normal(size=(4, 3))
    _, grads = mlp.loss_and_grad(params, x, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for e in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[e]
                flat[e] = old + h
                lp, _ = mlp.loss_and_grad(params, x, t)
                flat[e] = old - h
                lm, _ = mlp.loss_and_grad(params, x, t)
                flat[e] = old
                assert gf[e] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)


def test_adam_first_step_is_a_signed_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m1, v1 = mlp.adam(p, np.zeros(3), np.zeros(3), g, 1, 0.01)
    # m_hat = g, v_hat = g^2: the step is lr g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
