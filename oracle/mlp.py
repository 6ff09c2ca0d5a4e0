"""Multilayer perceptron of the learned warm start, FP64 NumPy.

TEST INFRASTRUCTURE ONLY (like the rest of this package).

The network maps a day's loads to an initial point of the solver: hidden
layers h_i = gelu(h_{i-1} W_i + b_i) with gelu(z) = z Phi(z), Phi the
standard normal distribution function, then a linear output layer
y = h_depth W_out + b_out.  The loss is the mean squared error over all
entries of a batch, L = sum (y - t)^2 / (batch * d_out), minimised by Adam
(beta1 0.9, beta2 0.999, eps 1e-8).  The reverse pass below is the chain rule
written out layer by layer.

Parameters are a list [(W_1, b_1), ..., (W_depth, b_depth), (W_out, b_out)]
with W_i shaped [fan_in, fan_out].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["gelu", "gelu_grad", "forward", "loss_and_grad", "adam"]

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * phi


def forward(params, x, keep=False):
    """Network output for a batch x [B, d_in]; with keep, also the
    pre-activations and activations of every hidden layer."""
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for W, b in params[:-1]:
        z = h @ W + b
        h = gelu(z)
        zs.append(z)
        hs.append(h)
    W, b = params[-1]
    y = h @ W + b
    return (y, zs, hs) if keep else y


def loss_and_grad(params, x, t):
    """Mean squared error and its gradient [(dW_i, db_i), ...]."""
    y, zs, hs = forward(params, x, keep=True)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    d = y - t
    loss = float((d * d).sum() / n)
    g = 2.0 * d / n                      # dL/dy
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        h_in = hs[i]
        grads[i] = (h_in.T @ g, g.sum(axis=0))
        if i == 0:
            break
        W = params[i][0]
        g = (g @ W.T) * gelu_grad(zs[i - 1])
    return loss, grads


def adam(p, m, v, g, it, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of arrays p, m, v with gradient g at 1-based step it."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    p = p - lr * (m / (1.0 - beta1 ** it)) / (np.sqrt(v / (1.0 - beta2 ** it)) + eps)
    return p, m, v
