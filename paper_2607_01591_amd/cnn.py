"""Binding of the warm-start network kernels (include/cnn.h) and the network built on
them: argument marshalling and orchestration only; every arithmetic step runs in the
HIP kernels of libmoc."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional

import numpy as np

from . import moc

_P = C.POINTER
_vp, _i32, _i64, _f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float

SIGNATURES = {
    "cnn_conv3x3_forward": [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp],
    "cnn_weights_for_dgrad": [_vp, _i32, _i32, _vp, _vp],
    "cnn_conv3x3_wgrad": [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp],
    "cnn_bias_grad": [_vp, _i64, _i32, _vp, _vp],
    "cnn_relu_backward": [_vp, _vp, _i64, _vp, _vp, _vp],
    "cnn_mse_grad": [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp],
    "cnn_mse_grad_noalloc": [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp],
    "cnn_adam": [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _i32, _vp, _vp],
    "cnn_to_bf16": [_vp, _i64, _vp, _vp],
    "cnn_material_features": [_vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp],
    "cnn_gather_rows": [_vp, _vp, _i64, _i32, _i32, _vp, _vp],
    "cnn_gather_log": [_vp, _vp, _i64, _i32, _i32, _vp, _vp],
    "cnn_bilinear_sample": [_vp, _i32, _i32, _i32, _i32, _vp, _i64, _i32, _vp, _vp],
    "cnn_center": [_vp, _i64, _i64, _i32, _i32, _vp],
    "cnn_d4_transform": [_vp, _i32, _i32, _i32, _i32, _vp, _vp],
    "cnn_d4_accumulate": [_vp, _i32, _i32, _i32, _i32, _f32, _vp, _vp],
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = moc.lib()
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = C.c_int
            fn.argtypes = args
        _lib = L
    return _lib


def _p(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _s(stream=None):
    import torch
    return (torch.cuda.current_stream() if stream is None else stream).cuda_stream


def _ok(rc, what):
    if rc != 0:
        raise moc.MocError(rc, what)


# bfloat16 tensors are handled as torch.bfloat16 (same bit layout as the kernels' uint16)
def conv3x3(x, w, bias=None, relu=False, out_bf16=None, out_f32=None, stream=None, dilation=1):
    N, H, W, Ci = x.shape
    Co = w.shape[0]
    _ok(lib().cnn_conv3x3_forward(_p(x), _p(w), _p(bias), N, H, W, Ci, Co, int(dilation), int(relu), _p(out_bf16),
                                  _p(out_f32), _s(stream)), "cnn_conv3x3_forward")


def weights_for_dgrad(w_f32, out_bf16, stream=None):
    Co, _, Ci = w_f32.shape
    _ok(lib().cnn_weights_for_dgrad(_p(w_f32), Co, Ci, _p(out_bf16), _s(stream)), "cnn_weights_for_dgrad")


def wgrad(x, dz, dw, stream=None, dilation=1):
    N, H, W, Ci = x.shape
    Co = dz.shape[-1]
    _ok(lib().cnn_conv3x3_wgrad(_p(x), _p(dz), N, H, W, Ci, Co, int(dilation), _p(dw), _s(stream)),
        "cnn_conv3x3_wgrad")


def bias_grad(dz_f32, db, stream=None):
    Co = dz_f32.shape[-1]
    _ok(lib().cnn_bias_grad(_p(dz_f32), dz_f32.numel() // Co, Co, _p(db), _s(stream)), "cnn_bias_grad")


def relu_backward(dy, y_bf16, dz_f32=None, dz_bf16=None, stream=None):
    _ok(lib().cnn_relu_backward(_p(dy), _p(y_bf16), dy.numel(), _p(dz_f32), _p(dz_bf16), _s(stream)),
        "cnn_relu_backward")


def mse_grad(y, t, cv, dy, partials, stream=None):
    cs = y.shape[-1]
    _ok(lib().cnn_mse_grad(_p(y), _p(t), y.numel() // cs, cs, cv, _p(dy), _p(partials), _s(stream)),
        "cnn_mse_grad")


def mse_grad_noalloc(y, t, cv, dy, loss, stream=None):
    """cnn_mse_grad_noalloc: dy as mse_grad, loss (device FP64 [1]) = the mean squared error."""
    cs = y.shape[-1]
    _ok(lib().cnn_mse_grad_noalloc(_p(y), _p(t), y.numel() // cs, cs, cv, _p(dy), _p(loss), _s(stream)),
        "cnn_mse_grad_noalloc")


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, p_bf16=None, stream=None):
    _ok(lib().cnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, int(step), _p(p_bf16),
                       _s(stream)), "cnn_adam")


def to_bf16(src, dst, stream=None):
    _ok(lib().cnn_to_bf16(_p(src), src.numel(), _p(dst), _s(stream)), "cnn_to_bf16")


def material_features(sigma_t, sigma_s, nu_sigma_f, chi, out, stream=None):
    """out [M, 4 G] FP32 from FP64 device cross sections (see cnn_material_features)."""
    M, G = sigma_t.shape
    _ok(lib().cnn_material_features(_p(sigma_t), _p(sigma_s), _p(nu_sigma_f), _p(chi), M, G, _p(out), _s(stream)),
        "cnn_material_features")


def gather_rows(table, idx, Cp, out, stream=None):
    _ok(lib().cnn_gather_rows(_p(table), _p(idx), idx.numel(), table.shape[-1], Cp, _p(out), _s(stream)),
        "cnn_gather_rows")


def gather_log(table, idx, Cp, out, stream=None):
    _ok(lib().cnn_gather_log(_p(table), _p(idx), idx.numel(), table.shape[-1], Cp, _p(out), _s(stream)),
        "cnn_gather_log")


def center(img, C_used, stream=None):
    """In place: subtract each image's mean over pixels and channels [0, C_used)."""
    n = img.shape[0]
    npix = img.numel() // (n * img.shape[-1])
    _ok(lib().cnn_center(_p(img), n, npix, C_used, img.shape[-1], _s(stream)), "cnn_center")


def d4_transform(x, op, out, stream=None):
    """out = x under square symmetry op (0..7); BF16 [N, S, S, C]."""
    N, S, S2, Cc = x.shape
    if S != S2:
        raise ValueError("square images only")
    _ok(lib().cnn_d4_transform(_p(x), N, S, Cc, int(op), _p(out), _s(stream)), "cnn_d4_transform")


def d4_accumulate(y, C_used, op, weight, acc, stream=None):
    """acc += weight * (y mapped back from symmetry op); FP32 [S, S, Cs]."""
    S, S2, Cs = y.shape
    _ok(lib().cnn_d4_accumulate(_p(y), S, Cs, C_used, int(op), float(weight), _p(acc), _s(stream)),
        "cnn_d4_accumulate")


def bilinear(img, C_used, uv, out, apply_exp=True, stream=None):
    H, W, Cs = img.shape[-3:]
    _ok(lib().cnn_bilinear_sample(_p(img), H, W, Cs, C_used, _p(uv), uv.shape[0], int(apply_exp), _p(out),
                                  _s(stream)), "cnn_bilinear_sample")


class ConvNet:
    """L-layer 3x3 network (ReLU between layers, linear output) on the HIP kernels.

    chans: channel counts [C0, C1, ..., CL] already padded (C0..C_{L-1} multiples of 32,
    CL a multiple of 32 as well so that the input gradient of the last layer can reuse
    the forward kernel). dilations: per layer (default 1). Master weights are FP32; BF16
    copies feed the matrix cores.
    """

    def __init__(self, chans: List[int], device, seed: int = 0, in_used: Optional[int] = None,
                 out_used: Optional[int] = None, dilations: Optional[List[int]] = None):
        import torch
        self.chans = chans
        self.dil = list(dilations) if dilations is not None else [1] * (len(chans) - 1)
        if len(self.dil) != len(chans) - 1:
            raise ValueError("one dilation per layer")
        self.dev = device
        g = np.random.default_rng(seed)
        self.W, self.b, self.Wb = [], [], []
        for li, (ci, co) in enumerate(zip(chans[:-1], chans[1:])):
            ci_used = in_used if (li == 0 and in_used) else ci
            co_used = out_used if (li == len(chans) - 2 and out_used) else co
            w = np.zeros((co, 9, ci), np.float32)
            std = np.sqrt(2.0 / (9 * ci_used))
            w[:co_used, :, :ci_used] = g.normal(0, std, size=(co_used, 9, ci_used))
            self.W.append(torch.tensor(w, device=device))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=device))
            self.Wb.append(torch.empty((co, 9, ci), dtype=torch.bfloat16, device=device))
        self._sync_bf16()
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0
        self.co_masks = [None] * len(self.W)
        self.out_used = out_used or chans[-1]

    def _sync_bf16(self):
        for w, wb in zip(self.W, self.Wb):
            to_bf16(w, wb)

    def forward(self, x, keep=False):
        """x: BF16 [N, H, W, C0]. Returns the FP32 output [N, H, W, CL] (and the list of
        BF16 layer inputs when keep)."""
        import torch
        N, H, Wd, _ = x.shape
        acts = [x]
        h = x
        L = len(self.W)
        out = None
        for li in range(L):
            co = self.chans[li + 1]
            if li < L - 1:
                nxt = torch.empty((N, H, Wd, co), dtype=torch.bfloat16, device=self.dev)
                conv3x3(h, self.Wb[li], self.b[li], relu=True, out_bf16=nxt, dilation=self.dil[li])
                acts.append(nxt)
                h = nxt
            else:
                out = torch.empty((N, H, Wd, co), dtype=torch.float32, device=self.dev)
                conv3x3(h, self.Wb[li], self.b[li], relu=False, out_f32=out, dilation=self.dil[li])
        return (out, acts) if keep else out

    def gradients(self, x, target, cv):
        """Loss and (dW, db) of MSE(forward(x)[..., :cv], target[..., :cv])."""
        import torch
        y, acts = self.forward(x, keep=True)
        N, H, Wd, _ = x.shape
        dy = torch.empty_like(y)
        parts = torch.zeros(256, dtype=torch.float64, device=self.dev)
        mse_grad(y, target, cv, dy, parts)
        L = len(self.W)
        dz_f = dy
        dz_b = torch.empty(dy.shape, dtype=torch.bfloat16, device=self.dev)
        to_bf16(dz_f, dz_b)
        grads = [None] * L
        for li in reversed(range(L)):
            dW = torch.zeros_like(self.W[li])
            db = torch.zeros_like(self.b[li])
            wgrad(acts[li], dz_b, dW, dilation=self.dil[li])
            bias_grad(dz_f, db)
            grads[li] = (dW, db)
            if li > 0:
                wt = torch.empty((self.chans[li], 9, self.chans[li + 1]), dtype=torch.bfloat16, device=self.dev)
                weights_for_dgrad(self.W[li], wt)
                dx = torch.empty((N, H, Wd, self.chans[li]), dtype=torch.float32, device=self.dev)
                conv3x3(dz_b, wt, None, relu=False, out_f32=dx, dilation=self.dil[li])
                dz_f = torch.empty_like(dx)
                dz_b = torch.empty(dx.shape, dtype=torch.bfloat16, device=self.dev)
                relu_backward(dx, acts[li], dz_f, dz_b)
        loss = float(parts.sum().item()) / (y.numel() // y.shape[-1] * cv)
        return loss, grads

    def apply(self, grads, lr=1e-3):
        self.step += 1
        for li, (dW, db) in enumerate(grads):
            adam(self.W[li], dW, self.mW[li], self.vW[li], self.step, lr=lr, p_bf16=self.Wb[li])
            adam(self.b[li], db, self.mb[li], self.vb[li], self.step, lr=lr)

    def train_step(self, x, target, cv, lr=1e-3):
        """One Adam step; returns the loss before the step."""
        loss, grads = self.gradients(x, target, cv)
        self.apply(grads, lr)
        return loss

    def state(self):
        return {"W": [w.cpu().numpy() for w in self.W], "b": [b.cpu().numpy() for b in self.b],
                "chans": list(self.chans), "dil": list(self.dil)}

    def load(self, st):
        import torch
        for i, (w, b) in enumerate(zip(st["W"], st["b"])):
            self.W[i].copy_(torch.as_tensor(w))
            self.b[i].copy_(torch.as_tensor(b))
        self._sync_bf16()
