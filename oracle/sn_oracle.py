"""ctypes wrapper around the plain-C FP64 DFEM-SN oracle (``dfem_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

Angular quadrature (a reading; the paper names only "discrete ordinates"): the product
of A equally spaced azimuths phi_a = 2 pi (a + 1/2) / A over [0, 2 pi) and the P
half-range Gauss-Legendre polar cosines of the planar oracle; for a planar problem each
in-plane direction (sin(theta_p) cos(phi_a), sin(theta_p) sin(phi_a)) stands for +-mu_p,
weight 4 pi w_p / A (the weights sum to 4 pi). Direction index d = a P + p. The mirror of
direction (a, p) across a side normal to x is (A/2 - 1 - a mod A, p), across a side
normal to y (A - 1 - a, p).

Array conventions: moments [T, G, 3] per triangle (modal coefficients of 1,
(x - x_c)/L, (y - y_c)/L with L = sqrt(area)), angular flux [nd, T, G, 3].
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

from .oracle import _f64, _i32, _p, polar_gl

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdfemoracle.so")
_SRC = os.path.join(_HERE, "dfem_oracle.c")


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO



def build_sanitized(out: str) -> str:
    """The same source built for a sanitizer run (tests only): AddressSanitizer and
    UndefinedBehaviorSanitizer, the process preloading gcc's libasan."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", out, _SRC, "-lm"])
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.POINTER
        d, i, v = C.c_double, C.c_int, C.c_void_p
        L.dfo_create.restype = v
        L.dfo_create.argtypes = [i, P(d), i, P(i), P(i), P(i), P(d), P(i), i, i, P(d), P(d), P(d), P(d),
                                 i, P(d), P(d), P(d), P(i), P(i)]
        L.dfo_destroy.argtypes = [v]
        L.dfo_info.argtypes = [v, P(i)]
        L.dfo_geometry.argtypes = [v, P(d), P(d), P(i), P(i)]
        L.dfo_get_psi.argtypes = [v, P(d)]
        L.dfo_set_external_source.argtypes = [v, P(d)]
        L.dfo_sweep.argtypes = [v, P(d), P(d)]
        L.dfo_sweep_linear.argtypes = [v, i, P(d), P(d), d, d, d, P(d)]
        L.dfo_emission.argtypes = [v, P(d), d, P(d)]
        L.dfo_solve.restype = i
        L.dfo_solve.argtypes = [v, d, i, P(d), P(d), P(i), P(d), P(d), i]
        _lib = L
    return _lib


def directions(A: int, P: int):
    """(mux, muy, w, rx, ry) of the product quadrature described in the module doc."""
    mu, wp = polar_gl(P)
    s = np.sqrt(1.0 - mu * mu)
    n = A * P
    mux, muy, w = np.zeros(n), np.zeros(n), np.zeros(n)
    rx, ry = np.zeros(n, np.int32), np.zeros(n, np.int32)
    for a in range(A):
        phi = 2.0 * math.pi * (a + 0.5) / A
        for p in range(P):
            d = a * P + p
            mux[d], muy[d] = s[p] * math.cos(phi), s[p] * math.sin(phi)
            w[d] = 4.0 * math.pi * wp[p] / A
            rx[d] = ((A // 2 - 1 - a) % A) * P + p
            ry[d] = (A - 1 - a) * P + p
    return mux, muy, w, rx, ry


class SNOracle:
    """FP64 DFEM-SN reference for a planar box problem (``problems.Problem``): every
    triangle is an element; A azimuths (default: the problem's n_azim) x P polar."""

    def __init__(self, prob, n_azim: int | None = None, n_polar: int | None = None):
        A = int(n_azim or prob.n_azim)
        Pn = int(n_polar or prob.n_polar)
        mux, muy, w, rx, ry = directions(A, Pn)
        self.nd, self.T, self.G = len(w), len(prob.tri), prob.n_groups
        self.w = w
        self._keep = [_f64(prob.xy), _i32(prob.tri), _i32(prob.tri_region), _i32(prob.region_material),
                      _f64(prob.box), _i32(np.asarray(prob.bc)[:4]), _f64(prob.sigma_t), _f64(prob.sigma_s),
                      _f64(prob.nu_sigma_f), _f64(prob.chi), _f64(mux), _f64(muy), _f64(w), _i32(rx), _i32(ry)]
        xy, tri, tr, rm, box, bc, st, ss, nsf, chi, mx, my, ww, rxa, rya = self._keep
        M = st.shape[0]
        h = lib().dfo_create(len(xy), _p(xy, C.c_double), len(tri), _p(tri, C.c_int), _p(tr, C.c_int),
                             _p(rm, C.c_int), _p(box, C.c_double), _p(bc, C.c_int), M, self.G, _p(st, C.c_double),
                             _p(ss, C.c_double), _p(nsf, C.c_double), _p(chi, C.c_double), self.nd,
                             _p(mx, C.c_double), _p(my, C.c_double), _p(ww, C.c_double), _p(rxa, C.c_int),
                             _p(rya, C.c_int))
        self._h = C.c_void_p(h)
        info = np.zeros(2, np.int32)
        lib().dfo_info(self._h, _p(info, C.c_int))
        self.n_levels = int(info[0])
        self.nu_sigma_f = nsf
        self._qext = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dfo_destroy(h)
            self._h = None

    def shape(self):
        return (self.T, self.G, 3)

    def geometry(self):
        area = np.zeros(self.T)
        mass = np.zeros((self.T, 3, 3))
        nbr = np.zeros((self.T, 3), np.int32)
        level = np.zeros((self.nd, self.T), np.int32)
        lib().dfo_geometry(self._h, _p(area, C.c_double), _p(mass, C.c_double), _p(nbr, C.c_int), _p(level, C.c_int))
        return dict(area=area, mass=mass, nbr=nbr, level=level)

    def get_psi(self):
        a = np.zeros((self.nd, self.T, self.G, 3))
        lib().dfo_get_psi(self._h, _p(a, C.c_double))
        return a

    def set_external_source(self, q):
        if q is None:
            self._qext = None
            lib().dfo_set_external_source(self._h, None)
        else:
            self._qext = _f64(q).reshape(self.shape())
            lib().dfo_set_external_source(self._h, _p(self._qext, C.c_double))

    def sweep(self, src):
        s = _f64(src).reshape(self.shape())
        phi = np.zeros(self.shape())
        lib().dfo_sweep(self._h, _p(s, C.c_double), _p(phi, C.c_double))
        return phi

    def sweep_linear(self, d, sigma_t, q, a, b, c):
        """One direction with a per-element linear source (per steradian, modal [T, 3]),
        Sigma_t per element, and the linear inflow a + b x + c y on every boundary face."""
        st = _f64(sigma_t).reshape(self.T)
        qq = _f64(q).reshape(self.T, 3)
        psi = np.zeros((self.T, 3))
        lib().dfo_sweep_linear(self._h, int(d), _p(st, C.c_double), _p(qq, C.c_double), float(a), float(b), float(c),
                               _p(psi, C.c_double))
        return psi

    def emission(self, phi, k):
        ph = _f64(phi).reshape(self.shape())
        out = np.zeros(self.shape())
        lib().dfo_emission(self._h, _p(ph, C.c_double), float(k), _p(out, C.c_double))
        return out

    def solve(self, tol=1e-6, max_iter=10000, phi0=None, k0=1.0, eigen=None):
        if eigen is None:
            eigen = bool(np.any(self.nu_sigma_f > 0)) and self._qext is None
        if phi0 is None:
            phi = np.zeros(self.shape())
            phi[..., 0] = 1.0
        else:
            phi = _f64(phi0).reshape(self.shape()).copy()
        k = C.c_double(k0)
        it = C.c_int()
        res, dk = C.c_double(), C.c_double()
        rc = lib().dfo_solve(self._h, tol, max_iter, _p(phi, C.c_double), C.byref(k), C.byref(it), C.byref(res),
                             C.byref(dk), int(eigen))
        return dict(phi=phi, k=k.value, iterations=it.value, residual=res.value, dk=dk.value, converged=(rc == 0))
