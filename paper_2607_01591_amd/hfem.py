"""Python binding of libmoc's diffusion HFEM solver (include/hfem.h): argument marshalling only.

Every step runs in libmoc's host checks, device preassembly and HIP kernels; this module
converts a ``problems.BrickGrid`` and torch device tensors into the C structures and
pointers of the ABI. There is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import moc
from .moc import (MOC_ENOCONV, MOC_OK, MocError, MocProfile, MocResult, MocXS, _dptr, _f64, _i32, _i64, _P, _ptr,
                  _stream_handle)


class MocHfemGrid(C.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("x_edges", _P(_f64)), ("y_edges", _P(_f64)),
                ("z_edges", _P(_f64)), ("node_material", _P(_i32)), ("bc", _i32 * 6)]


class MocHfemOptions(C.Structure):
    _fields_ = [("volume_order", _i32), ("face_order", _i32), ("inner_iterations", _i32), ("max_iter", _i32),
                ("device", _i32), ("check_every", _i32), ("fp32_matrices", _i32)]


class MocHfemInfo(C.Structure):
    _fields_ = [("n_nodes", _i32), ("n_groups", _i32), ("n_moments", _i32), ("n_face_dofs", _i32), ("n_red", _i32),
                ("n_black", _i32), ("inner_iterations", _i32), ("device_bytes", _i64), ("setup_ms", _f64),
                ("assemble_ms", _f64), ("fp32_matrices", _i32)]


SIGNATURES = {
    "moc_hfem_create": (C.c_int, [_P(MocHfemGrid), _P(MocXS), _P(MocHfemOptions), _P(C.c_void_p)]),
    "moc_hfem_destroy": (None, [C.c_void_p]),
    "moc_hfem_sweep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_hfem_solve": (C.c_int, [C.c_void_p, _f64, _P(MocResult)]),
    "moc_hfem_run_iterations": (C.c_int, [C.c_void_p, _i32, _P(MocResult)]),
    "moc_hfem_get_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_hfem_get_currents": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_hfem_set_external_source": (C.c_int, [C.c_void_p, C.c_void_p]),
    "moc_hfem_get_info": (C.c_int, [C.c_void_p, _P(MocHfemInfo)]),
    "moc_hfem_set_profiling": (C.c_int, [C.c_void_p, _i32]),
    "moc_hfem_get_profile": (C.c_int, [C.c_void_p, _P(MocProfile)]),
    "moc_hfem_last_error": (C.c_char_p, [C.c_void_p]),
}

_ready = False


def lib():
    global _ready
    L = moc.lib()
    if not _ready:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


def make_structs(grid, volume_order=2, face_order=1, inner_iterations=2, max_iter=10000, device=0, check_every=1,
                 fp32_matrices=False):
    """The ABI structures of a BrickGrid; returns (grid, xs, options, keep-alive list)."""
    keep = []

    def k(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    ex, ey, ez = (k(e, np.float64) for e in grid.edges)
    nm = k(grid.node_material, np.int32)
    g = MocHfemGrid()
    g.nx, g.ny, g.nz = len(ex) - 1, len(ey) - 1, len(ez) - 1
    g.x_edges, g.y_edges, g.z_edges = _ptr(ex, _f64), _ptr(ey, _f64), _ptr(ez, _f64)
    g.node_material = _ptr(nm, _i32)
    for i, b in enumerate(grid.bc):
        g.bc[i] = int(b)
    st, ss, nsf, chi = (k(a, np.float64) for a in (grid.sigma_t, grid.sigma_s, grid.nu_sigma_f, grid.chi))
    x = MocXS()
    x.n_materials, x.n_groups = st.shape
    x.sigma_t, x.sigma_s, x.nu_sigma_f, x.chi = _ptr(st, _f64), _ptr(ss, _f64), _ptr(nsf, _f64), _ptr(chi, _f64)
    o = MocHfemOptions(volume_order, face_order, inner_iterations, max_iter, device, check_every, int(fp32_matrices))
    return g, x, o, keep


class HFEMSolver:
    """One HFEM context for a ``problems.BrickGrid``; flux and source tensors are device
    FP64 [N, G, Np] in node order, partial currents [N, G, Nft]. fp32_matrices stores R and
    A^-1 in FP32 (FP64 arithmetic otherwise unchanged)."""

    def __init__(self, grid, volume_order: int = 2, face_order: int = 1, inner_iterations: int = 2,
                 max_iter: int = 10000, device: int = 0, check_every: int = 1, fp32_matrices: bool = False):
        L = lib()
        g, x, o, keep = make_structs(grid, volume_order, face_order, inner_iterations, max_iter, device, check_every,
                                     fp32_matrices)
        h = C.c_void_p()
        rc = L.moc_hfem_create(C.byref(g), C.byref(x), C.byref(o), C.byref(h))
        del keep
        if rc != MOC_OK:
            raise MocError(rc, L.moc_hfem_last_error(None).decode())
        self._h = h
        self.device = device
        inf = MocHfemInfo()
        L.moc_hfem_get_info(self._h, C.byref(inf))
        self.info = {f: getattr(inf, f) for f, _ in MocHfemInfo._fields_}
        self.N, self.G = self.info["n_nodes"], self.info["n_groups"]
        self.Np, self.Nft = self.info["n_moments"], self.info["n_face_dofs"]

    def close(self):
        if getattr(self, "_h", None) is not None and moc is not None and moc._lib is not None:
            moc._lib.moc_hfem_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, ok=(MOC_OK,)):
        if rc not in ok:
            raise MocError(rc, lib().moc_hfem_last_error(self._h).decode())
        return rc

    def shape(self):
        return (self.N, self.G, self.Np)

    def sweep(self, source, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape(), dtype=torch.float64, device=source.device)
        self._check(lib().moc_hfem_sweep(self._h, _dptr(source), _dptr(out), _stream_handle(stream)))
        return out

    def solve(self, tol: float = 1e-6, raise_on_noconv: bool = False) -> dict:
        import torch
        torch.cuda.current_stream().synchronize()
        r = MocResult()
        rc = lib().moc_hfem_solve(self._h, tol, C.byref(r))
        self._check(rc, (MOC_OK,) if raise_on_noconv else (MOC_OK, MOC_ENOCONV))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk, wall_ms=r.wall_ms,
                    sweeps=r.sweeps, converged=(rc == MOC_OK))

    def run_iterations(self, n: int) -> dict:
        import torch
        torch.cuda.current_stream().synchronize()
        r = MocResult()
        self._check(lib().moc_hfem_run_iterations(self._h, int(n), C.byref(r)))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk, wall_ms=r.wall_ms)

    def flux(self, stream=None):
        import torch
        out = torch.empty(self.shape(), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().moc_hfem_get_flux(self._h, _dptr(out), _stream_handle(stream)))
        return out

    def currents(self, stream=None):
        import torch
        out = torch.empty((self.N, self.G, self.Nft), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().moc_hfem_get_currents(self._h, _dptr(out), _stream_handle(stream)))
        return out

    def set_external_source(self, q):
        import torch
        if q is None:
            self._check(lib().moc_hfem_set_external_source(self._h, None))
            return
        torch.cuda.current_stream().synchronize()
        self._check(lib().moc_hfem_set_external_source(self._h, _dptr(q.contiguous())))

    def set_profiling(self, enable: bool = True):
        self._check(lib().moc_hfem_set_profiling(self._h, int(enable)))

    def profile(self) -> dict:
        p = MocProfile()
        self._check(lib().moc_hfem_get_profile(self._h, C.byref(p)))
        return dict(sweeps=p.sweeps, sweep_ms=p.sweep_ms, sweep_ms_min=p.sweep_ms_min, sweep_ms_max=p.sweep_ms_max)
