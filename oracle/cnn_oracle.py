"""FP64 numpy reference of the warm-start convolutional network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests to check the HIP BF16 kernels; the
product never imports it.

Network: L layers of 3x3 convolutions with zero padding ("same"), stride 1, NHWC
activations; ReLU after every layer but the last. Weights are stored as
W[co][ky][kx][ci] with bias b[co]. Loss: mean squared error over all outputs.

Every function is written from the definition of a discrete convolution:
    z[n, y, x, co] = b[co] + sum_{ky, kx, ci} x[n, y + ky - 1, x + kx - 1, ci] W[co, ky, kx, ci]
with x = 0 outside the image. Backward passes follow the chain rule term by term.
Pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv_forward(x, W, b):
    """x [N, H, Wd, Ci], W [Co, 3, 3, Ci], b [Co] -> z [N, H, Wd, Co]."""
    N, H, Wd, _ = x.shape
    xp = pad(x)
    z = np.zeros((N, H, Wd, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + Wd, :]           # x[n, y+ky-1, x+kx-1, :]
            z += patch @ W[:, ky, kx, :].T
    return z


def conv_backward(x, W, dz):
    """Gradients of conv_forward given dL/dz: returns (dx, dW, db)."""
    N, H, Wd, _ = x.shape
    xp = pad(x)
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + Wd, :]
            dW[:, ky, kx, :] = np.einsum("nyxo,nyxi->oi", dz, patch)
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dz @ W[:, ky, kx, :]
    db = dz.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dW, db


def forward(x, params):
    """params: list of (W, b). Returns the output and the per-layer inputs/pre-activations."""
    acts, pre = [x], []
    h = x
    for i, (W, b) in enumerate(params):
        z = conv_forward(h, W, b)
        pre.append(z)
        h = np.maximum(z, 0.0) if i < len(params) - 1 else z
        acts.append(h)
    return h, acts, pre


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, acts, pre, t):
    """Gradients of mse(forward(x), t) with respect to every (W, b)."""
    y = acts[-1]
    dh = 2.0 * (y - t) / y.size
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        dz = dh if i == len(params) - 1 else dh * (pre[i] > 0)
        dx, dW, db = conv_backward(acts[i], params[i][0], dz)
        grads[i] = (dW, db)
        dh = dx
    return grads


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place on copies; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
