"""Timing of the warm-start network's kernels at its real shape.

    python -m paper_2310_06650_amd.mlp_bench [--steps 50]

The network of the learned warm start (617-bus x 18-period loads and reserves
in, 3 x 512 GELU, every variable of the grid out; batch 64) with seeded
random weights and data: mean milliseconds of one FP32 training step (forward,
reverse, Adam) and of one BF16 forward, after warmup, as one JSON line with
the products' flops and the bytes the step must move at least (weights,
gradients, Adam moments).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import qg

D_IN, WIDTH, DEPTH, D_OUT, BATCH = 11124, 512, 3, 29412, 64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    args = ap.parse_args()
    import torch
    net = qg.MLP(D_IN, WIDTH, DEPTH, D_OUT, max_batch=BATCH)
    rng = np.random.default_rng(1)
    flat = np.zeros(net.n_params, dtype=np.float32)
    sizes = [D_IN] + [WIDTH] * DEPTH + [D_OUT]
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        wo, _ = net.offsets(i)
        flat[wo:wo + a * b] = rng.normal(0, 1.0 / np.sqrt(a), a * b).astype(np.float32)
    net.set_params(flat)
    x = torch.from_numpy(rng.normal(size=(BATCH, D_IN)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=(BATCH, D_OUT)).astype(np.float32)).cuda()
    for _ in range(3):
        net.train_step(x, t, 1e-4)
        net.forward_bf16(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    train_s = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward_bf16(x)
    torch.cuda.synchronize()
    fwd_s = (time.perf_counter() - t0) / args.steps
    macs = sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    fwd_flop = 2 * BATCH * macs
    # forward, activation gradients (all but the first layer) and weight gradients
    train_flop = fwd_flop + 2 * BATCH * (macs - D_IN * WIDTH) + 2 * BATCH * macs
    n = net.n_params
    # weights read by the forward and the activation gradients, gradient written,
    # Adam: parameters, gradient and both moments read, parameters and moments written
    train_bytes = 4 * (n + (n - D_IN * WIDTH) + n + 7 * n)
    out = dict(shape=f"{D_IN}-{WIDTH}x{DEPTH}-{D_OUT}, batch {BATCH}", params=int(n),
               steps=args.steps, train_step_ms=train_s * 1e3, bf16_forward_ms=fwd_s * 1e3,
               train_tflops=train_flop / train_s / 1e12, bf16_forward_tflops=fwd_flop / fwd_s / 1e12,
               train_min_bytes=int(train_bytes), train_gbps=train_bytes / train_s / 1e9)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
