"""FP64 numpy reference of the warm-start convolutional network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests to check the HIP BF16 kernels; the
product never imports it.

Network: L layers of 3x3 convolutions with zero padding ("same"), stride 1, NHWC
activations; ReLU after every layer but the last. Weights are stored as
W[co][ky][kx][ci] with bias b[co]. Loss: mean squared error over all outputs.

Every function is written from the definition of a discrete (dilated) convolution:
    z[n, y, x, co] = b[co] + sum_{ky, kx, ci} x[n, y + (ky - 1) d, x + (kx - 1) d, ci] W[co, ky, kx, ci]
with x = 0 outside the image and dilation d >= 1 (d = 1: the plain 3x3 convolution).
Backward passes follow the chain rule term by term. Pinned by central finite
differences and, for d > 1, by the polyphase identity (a dilated convolution acts on
each of the d x d interleaved sub-images as the plain convolution) in the tests.
"""
from __future__ import annotations

import numpy as np


def pad(x, d=1):
    return np.pad(x, ((0, 0), (d, d), (d, d), (0, 0)))


def conv_forward(x, W, b, d=1):
    """x [N, H, Wd, Ci], W [Co, 3, 3, Ci], b [Co] -> z [N, H, Wd, Co]; dilation d."""
    N, H, Wd, _ = x.shape
    xp = pad(x, d)
    z = np.zeros((N, H, Wd, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky * d:ky * d + H, kx * d:kx * d + Wd, :]   # x[n, y+(ky-1)d, x+(kx-1)d, :]
            z += patch @ W[:, ky, kx, :].T
    return z


def conv_backward(x, W, dz, d=1):
    """Gradients of conv_forward given dL/dz: returns (dx, dW, db)."""
    N, H, Wd, _ = x.shape
    xp = pad(x, d)
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky * d:ky * d + H, kx * d:kx * d + Wd, :]
            dW[:, ky, kx, :] = np.einsum("nyxo,nyxi->oi", dz, patch)
            dxp[:, ky * d:ky * d + H, kx * d:kx * d + Wd, :] += dz @ W[:, ky, kx, :]
    db = dz.sum(axis=(0, 1, 2))
    return dxp[:, d:d + H, d:d + Wd, :], dW, db


def forward(x, params, dils=None):
    """params: list of (W, b); dils: dilation per layer (default 1). Returns the output
    and the per-layer inputs/pre-activations."""
    dils = dils or [1] * len(params)
    acts, pre = [x], []
    h = x
    for i, (W, b) in enumerate(params):
        z = conv_forward(h, W, b, dils[i])
        pre.append(z)
        h = np.maximum(z, 0.0) if i < len(params) - 1 else z
        acts.append(h)
    return h, acts, pre


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, acts, pre, t, dils=None):
    """Gradients of mse(forward(x), t) with respect to every (W, b)."""
    dils = dils or [1] * len(params)
    y = acts[-1]
    dh = 2.0 * (y - t) / y.size
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        dz = dh if i == len(params) - 1 else dh * (pre[i] > 0)
        dx, dW, db = conv_backward(acts[i], params[i][0], dz, dils[i])
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


def material_features(sigma_t, sigma_s, nu_sigma_f, chi):
    """Input features of the warm-start network per material, [M, 4 G] FP64: the log of
    the normalised infinite-medium spectrum phi, which balances removal by collision
    against in-scattering and the fission spectrum, Sigma_t,g phi_g - sum_g' Sigma_s,g'->g
    phi_g' = chi_g (sigma_s[m][g][g'] scatters from g to g'); a material without
    fission takes the mean chi of the fissile ones (1/G if there are none); |phi| is
    floored at 1e-30 before normalising to sum 1. Then Sigma_t, Sigma_a = Sigma_t minus
    the total scattering out of each group, and nuSigma_f."""
    st, ss, nsf, chi = (np.asarray(a, np.float64) for a in (sigma_t, sigma_s, nu_sigma_f, chi))
    M, G = st.shape
    fissile = nsf.sum(axis=1) > 0
    chi_free = chi[fissile].mean(axis=0) if fissile.any() else np.full(G, 1.0 / G)
    out = np.zeros((M, 4 * G))
    for m in range(M):
        removal = np.diag(st[m]) - ss[m].T            # row g: collisions minus in-scatter
        phi = np.linalg.solve(removal, chi[m] if fissile[m] else chi_free)
        phi = np.maximum(np.abs(phi), 1e-30)
        out[m, :G] = np.log(phi / phi.sum())
        out[m, G:2 * G] = st[m]
        out[m, 2 * G:3 * G] = st[m] - ss[m].sum(axis=1)
        out[m, 3 * G:] = nsf[m]
    return out
