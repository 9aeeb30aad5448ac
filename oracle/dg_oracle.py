"""ctypes wrapper around the plain-C FP64 DGMOC oracle (``dgmoc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package. The tracks, segments, links
and quadrature come from the planar oracle (``oracle.Oracle``), i.e. from the oracle's own
tracking, so nothing here depends on the product library.

Array conventions (all FP64, C order):
  * scalar-flux and emission moments: [Nz, R, G, 2], moment 1 = coefficient of the
    Legendre function xi on the plane (xi = -1 at the bottom face, +1 at the top);
  * radial boundary fluxes: [2 wards, Nz, T, 2 senses, P, G, 2], in each ward's local
    orientation (the downward ward mirrors xi);
  * bottom-face buffer: [NA, 2 senses, P, R, G].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .oracle import Oracle, _f64, _i32, _p

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdgoracle.so")
_SRC = os.path.join(_HERE, "dgmoc_oracle.c")


def build(force: bool = False) -> str:
    """Compile the DGMOC oracle with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
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
        d, i, i64, v = C.c_double, C.c_int, C.c_int64, C.c_void_p
        L.dgo_create.restype = v
        L.dgo_create.argtypes = [i, P(i), P(i64), P(i), P(d), P(i), i, P(d), P(d), i, P(d), P(d),
                                 i, i, i, P(d), P(d), P(d), P(d), i, P(d), P(i), i, i]
        L.dgo_destroy.argtypes = [v]
        L.dgo_volumes.argtypes = [v, P(d), P(d)]
        L.dgo_get_psi.argtypes = [v, P(d)]
        L.dgo_set_psi.argtypes = [v, P(d)]
        L.dgo_get_exit.argtypes = [v, P(d)]
        L.dgo_get_bottom.argtypes = [v, P(d)]
        L.dgo_set_external_source.argtypes = [v, P(d)]
        L.dgo_expm2.argtypes = [P(d), P(d)]
        L.dgo_segment.argtypes = [d, d, d, d, d, d, P(d), P(d), P(d)]
        L.dgo_sweep.argtypes = [v, P(d), P(d), P(d)]
        L.dgo_emission.argtypes = [v, P(d), d, P(d)]
        L.dgo_solve.restype = i
        L.dgo_solve.argtypes = [v, d, i, P(d), P(d), P(i), P(d), P(d), i]
        _lib = L
    return _lib


def expm2(B):
    """e^B of a 2x2 matrix (the oracle's scaling-and-squaring series)."""
    b = _f64(B).reshape(4)
    e = np.zeros(4)
    lib().dgo_expm2(_p(b, C.c_double), _p(e, C.c_double))
    return e.reshape(2, 2)


def segment(sigma_t, kappa, f, q0, q1, psi_face, psi_in):
    """One segment of the 2x2 characteristic ODE: (psi_out, psi_bar)."""
    pin = _f64(psi_in).reshape(2)
    out, bar = np.zeros(2), np.zeros(2)
    lib().dgo_segment(float(sigma_t), float(kappa), float(f), float(q0), float(q1), float(psi_face),
                      _p(pin, C.c_double), _p(out, C.c_double), _p(bar, C.c_double))
    return out, bar


class DGOracle:
    """FP64 DGMOC reference for one extruded problem (``problems.Extruded``)."""

    def __init__(self, ext, planar: Oracle | None = None):
        base = ext.base
        o = planar if planar is not None else Oracle.from_problem(base)
        self.planar = o
        tr = o.tracks()
        reg, ln = o.segments()
        ang = o.angles()
        mu, wp = o.polar()
        self.T, self.NA, self.P, self.R, self.G = o.T, o.NA, o.P, o.R, o.G
        self.M = o.M
        self.Nz = int(len(ext.dz))
        self.dz = _f64(ext.dz)
        self.mu, self.wp = mu, wp
        self.angles = ang
        self.track_angle = tr["angle"]
        self._keep = [_i32(tr["angle"]), np.ascontiguousarray(tr["offset"], np.int64), _i32(reg), _f64(ln),
                      _i32(tr["link"]), _f64(ang["delta"]), _f64(ang["w"]), _f64(mu), _f64(wp),
                      _f64(base.sigma_t), _f64(base.sigma_s), _f64(base.nu_sigma_f), _f64(base.chi),
                      self.dz, _i32(ext.plane_material)]
        ta, off, rg, sl, lk, dl, wa, m_, w_, st, ss, nsf, chi, dz, mat = self._keep
        assert mat.shape == (self.Nz, self.R)
        h = lib().dgo_create(self.T, _p(ta, C.c_int), _p(off, C.c_int64), _p(rg, C.c_int), _p(sl, C.c_double),
                             _p(lk, C.c_int), self.NA, _p(dl, C.c_double), _p(wa, C.c_double), self.P,
                             _p(m_, C.c_double), _p(w_, C.c_double), self.R, self.M, self.G, _p(st, C.c_double),
                             _p(ss, C.c_double), _p(nsf, C.c_double), _p(chi, C.c_double), self.Nz,
                             _p(dz, C.c_double), _p(mat, C.c_int), int(ext.bc_bottom), int(ext.bc_top))
        self._h = C.c_void_p(h)
        self.plane_material = mat
        self.nu_sigma_f = nsf

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dgo_destroy(h)
            self._h = None

    # --- shapes and state -------------------------------------------------------------
    def flux_shape(self):
        return (self.Nz, self.R, self.G, 2)

    def psi_shape(self):
        return (2, self.Nz, self.T, 2, self.P, self.G, 2)

    def face_shape(self):
        return (self.NA, 2, self.P, self.R, self.G)

    def volumes(self):
        V, Va = np.zeros(self.R), np.zeros((self.NA, self.R))
        lib().dgo_volumes(self._h, _p(V, C.c_double), _p(Va, C.c_double))
        return V, Va

    def get_psi(self):
        a = np.zeros(self.psi_shape())
        lib().dgo_get_psi(self._h, _p(a, C.c_double))
        return a

    def set_psi(self, psi):
        a = _f64(np.broadcast_to(psi, self.psi_shape()))
        lib().dgo_set_psi(self._h, _p(a, C.c_double))

    def get_exit(self):
        a = np.zeros(self.psi_shape())
        lib().dgo_get_exit(self._h, _p(a, C.c_double))
        return a

    def get_bottom(self):
        a = np.zeros(self.face_shape())
        lib().dgo_get_bottom(self._h, _p(a, C.c_double))
        return a

    def set_external_source(self, q):
        if q is None:
            self._qext = None
            lib().dgo_set_external_source(self._h, None)
        else:
            self._qext = _f64(q).reshape(self.flux_shape())
            lib().dgo_set_external_source(self._h, _p(self._qext, C.c_double))

    # --- compute ------------------------------------------------------------------------
    def sweep(self, src, face_flow=False):
        """One sweep for emission moments src [Nz, R, G, 2]; returns phi (and, with
        face_flow, the axial inflow / outflow through the domain faces [2, G])."""
        s = _f64(src).reshape(self.flux_shape())
        phi = np.zeros(self.flux_shape())
        ff = np.zeros((2, self.G)) if face_flow else None
        lib().dgo_sweep(self._h, _p(s, C.c_double), _p(phi, C.c_double),
                        _p(ff, C.c_double) if ff is not None else None)
        return (phi, ff) if face_flow else phi

    def emission(self, phi, k):
        ph = _f64(phi).reshape(self.flux_shape())
        out = np.zeros(self.flux_shape())
        lib().dgo_emission(self._h, _p(ph, C.c_double), float(k), _p(out, C.c_double))
        return out

    def solve(self, tol=1e-6, max_iter=10000, phi0=None, k0=1.0, eigen=None):
        if eigen is None:
            eigen = bool(np.any(self.nu_sigma_f > 0)) and getattr(self, "_qext", None) is None
        if phi0 is None:
            phi = np.zeros(self.flux_shape())
            phi[..., 0] = 1.0
        else:
            phi = _f64(phi0).reshape(self.flux_shape()).copy()
        k = C.c_double(k0)
        it = C.c_int()
        res, dk = C.c_double(), C.c_double()
        rc = lib().dgo_solve(self._h, tol, max_iter, _p(phi, C.c_double), C.byref(k), C.byref(it),
                             C.byref(res), C.byref(dk), int(eigen))
        return dict(phi=phi, k=k.value, iterations=it.value, residual=res.value, dk=dk.value,
                    converged=(rc == 0))
