"""Learned warm start for the power iteration: rasterise a lattice's cross sections,
predict the scalar flux with the BF16 network (HIP matrix-core kernels), de-rasterise
it to the regions and hand it to moc_set_initial_guess. The plain iteration still
decides convergence; a rejected guess falls back to the cold start.

Image: 128 x 128 pixels over the lattice's bounding box. Input channels (per pixel,
from the material of the region containing the pixel centre): the log of the material's
infinite-medium spectrum, Sigma_t, Sigma_a and nuSigma_f for each of the 7 groups (28,
padded to 32). Output: log(phi) per group (7, padded to 32) up to one additive constant
per image (the solver rescales the guess).
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np

from . import cnn, moc

IMG = 128
C_IN, C_IN_PAD = 28, 32
C_OUT_PAD = 32
CHANNELS = [C_IN_PAD, 64, 64, 64, 64, 64, 64, C_OUT_PAD]   # 7 layers, 64 channels
# Dilations double up to 32 pixels, then a local output layer: the receptive field is
# 1 + 2 (1 + 2 + 4 + 8 + 16 + 32 + 1) = 129 pixels, the whole 128-pixel image, so the
# network can see the lattice-wide flux shape (the slowly decaying error of the power
# iteration), not only a pin's neighbourhood.
DILATIONS = [1, 2, 4, 8, 16, 32, 1]


def load_net(path, device, n_groups) -> cnn.ConvNet:
    """A network with the channel counts and dilations stored in a weights file
    (numpy .npz written by train_warmstart; files without dilations are undilated)."""
    st = np.load(path)
    chans = [int(c) for c in st["chans"]]
    dil = [int(d) for d in st["dil"]] if "dil" in st.files else [1] * (len(chans) - 1)
    net = cnn.ConvNet(chans, device, seed=0, in_used=C_IN, out_used=n_groups, dilations=dil)
    net.load({"W": [st[f"W{i}"] for i in range(len(chans) - 1)], "b": [st[f"b{i}"] for i in range(len(chans) - 1)]})
    return net


def material_features(prob, device):
    """Per-material input features [M, 4 G] (device FP32, computed by the
    cnn_material_features kernel): the log of the material's infinite-medium spectrum
    (the solution of (Sigma_t - Sigma_s^T) phi = chi, with the lattice's mean fission
    spectrum for materials that do not fission; normalised to sum 1), then Sigma_t,
    Sigma_a = Sigma_t - sum_g' Sigma_s,g->g' and nuSigma_f. The spectrum is the part of
    the flux a few pixels of context cannot infer from raw cross sections."""
    import torch
    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
    M, G = prob.sigma_t.shape
    out = torch.empty((M, 4 * G), dtype=torch.float32, device=device)
    cnn.material_features(dev(prob.sigma_t), dev(prob.sigma_s), dev(prob.nu_sigma_f), dev(prob.chi), out)
    return out


class WarmStart:
    """Raster maps for one mesh (shared by every problem on it) and the network."""

    def __init__(self, solver: "moc.Solver", prob, device, net: Optional[cnn.ConvNet] = None):
        import torch
        self.solver = solver
        self.dev = device
        self.G = prob.n_groups
        x0, y0, x1, y1 = prob.box
        self.dx, self.dy = (x1 - x0) / IMG, (y1 - y0) / IMG
        cx = x0 + (np.arange(IMG) + 0.5) * self.dx
        cy = y0 + (np.arange(IMG) + 0.5) * self.dy
        X, Y = np.meshgrid(cx, cy, indexing="xy")
        pix_region = solver.locate(np.stack([X.ravel(), Y.ravel()], 1))
        if (pix_region < 0).any():
            raise ValueError("warm start: a pixel centre lies outside the mesh")
        self.pix_region_host = pix_region
        self.pix_region = torch.as_tensor(pix_region, device=device)
        cen = solver.centroids()
        uv = np.stack([(cen[:, 0] - x0) / self.dx - 0.5, (cen[:, 1] - y0) / self.dy - 0.5], 1)
        self.uv = torch.as_tensor(uv.astype(np.float32), device=device)
        self.net = net if net is not None else cnn.ConvNet(CHANNELS, device, seed=0, in_used=C_IN,
                                                           out_used=self.G, dilations=DILATIONS)

    # ---------------------------------------------------------------- data
    def rasterize(self, prob, out=None):
        """BF16 input image [1, IMG, IMG, 32] of a problem on this mesh."""
        import torch
        table = material_features(prob, self.dev)
        idx = torch.as_tensor(prob.region_material[self.pix_region_host].astype(np.int32), device=self.dev)
        if out is None:
            out = torch.empty((1, IMG, IMG, C_IN_PAD), dtype=torch.bfloat16, device=self.dev)
        cnn.gather_rows(table, idx, C_IN_PAD, out)
        return out

    def target(self, phi_user, out=None):
        """FP32 target image [1, IMG, IMG, 32] = log(phi) of the region under each pixel."""
        import torch
        if out is None:
            out = torch.empty((1, IMG, IMG, C_OUT_PAD), dtype=torch.float32, device=self.dev)
        cnn.gather_log(phi_user, self.pix_region, C_OUT_PAD, out)
        return out

    def predict(self, prob, symmetrize: bool = True):
        """Predicted scalar flux [R, G] (device FP64, user order) and the time spent.
        symmetrize: average the network's log-flux over the 8 symmetries of the square
        lattice image (rotate / mirror the input, map each output back), which removes the
        part of the prediction error that does not respect the lattice's symmetry."""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        img = self.rasterize(prob)
        if symmetrize:
            out = torch.zeros((IMG, IMG, C_OUT_PAD), dtype=torch.float32, device=self.dev)
            t = torch.empty_like(img)
            for op in range(8):
                cnn.d4_transform(img, op, t)
                y = self.net.forward(t)
                cnn.d4_accumulate(y[0], self.G, op, 1.0 / 8.0, out)
        else:
            out = self.net.forward(img)[0]
        phi0 = torch.empty((self.solver.R, self.G), dtype=torch.float64, device=self.dev)
        cnn.bilinear(out, self.G, self.uv, phi0, apply_exp=True)
        torch.cuda.synchronize()
        return phi0, (time.perf_counter() - t0) * 1e3

    def solve_warm(self, prob, tol=1e-6, symmetrize: bool = True):
        """Warm-started solve: prediction + moc_solve; wall time includes the prediction."""
        phi0, pred_ms = self.predict(prob, symmetrize)
        self.solver.set_initial_guess(phi0, -1.0)
        r = self.solver.solve(tol)
        r["predict_ms"] = pred_ms
        r["total_ms"] = r["wall_ms"] + pred_ms
        return r


def homogenized_guess(prob, V, device):
    """Non-learned baseline: spatially flat flux with the infinite-medium spectrum of the
    volume-homogenised lattice (the dominant eigenvector of
    (diag Sigma_t - Sigma_s^T)^-1 chi nuSigma_f^T)."""
    import torch
    w = np.bincount(prob.region_material, weights=V, minlength=prob.n_materials)
    w = w / w.sum()
    st = w @ prob.sigma_t
    ss = np.tensordot(w, prob.sigma_s, axes=1)
    nsf = w @ prob.nu_sigma_f
    chi = w @ (prob.chi * (prob.nu_sigma_f.sum(axis=1, keepdims=True) > 0))
    chi = chi / chi.sum()
    spec = np.linalg.solve(np.diag(st) - ss.T, chi)
    spec = np.abs(spec)
    phi = np.broadcast_to(spec, (prob.n_regions, prob.n_groups)).copy()
    return torch.as_tensor(phi, device=device)
