"""Python binding of libmoc's DFEM-SN solver (include/dfem.h): argument marshalling only.

Every step runs in libmoc's host setup and HIP kernels; this module converts a planar
``problems.Problem`` (box domain) and torch device tensors into the C structures and
pointers of the ABI. There is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import moc
from .moc import (MOC_ENOCONV, MOC_OK, PREC, MocError, MocMesh, MocOptions, MocProfile, MocResult, MocTracks,
                  MocXS, _dptr, _f64, _i32, _i64, _P, _ptr, _stream_handle)


class MocSnInfo(C.Structure):
    _fields_ = [("n_elements", _i32), ("n_directions", _i32), ("n_groups", _i32), ("n_levels", _i32),
                ("n_tasks", _i64), ("n_slots", _i64), ("n_boundary_faces", _i64), ("device_bytes", _i64),
                ("setup_ms", _f64), ("tasks_per_thread", _i32), ("n_tiles", _i32), ("n_tile_levels", _i32),
                ("max_inner_levels", _i32), ("tile_lds_bytes", _i32), ("n_tile_slots", _i64)]


SIGNATURES = {
    "moc_sn_create": (C.c_int, [_P(MocMesh), _P(MocTracks), _P(MocXS), _P(MocOptions), _P(C.c_void_p)]),
    "moc_sn_destroy": (None, [C.c_void_p]),
    "moc_sn_sweep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_sn_solve": (C.c_int, [C.c_void_p, _f64, _P(MocResult)]),
    "moc_sn_run_iterations": (C.c_int, [C.c_void_p, _i32, _P(MocResult)]),
    "moc_sn_get_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_sn_set_external_source": (C.c_int, [C.c_void_p, C.c_void_p]),
    "moc_sn_get_info": (C.c_int, [C.c_void_p, _P(MocSnInfo)]),
    "moc_sn_set_tiles": (C.c_int, [C.c_void_p, _i32, C.c_void_p]),
    "moc_sn_set_profiling": (C.c_int, [C.c_void_p, _i32]),
    "moc_sn_get_profile": (C.c_int, [C.c_void_p, _P(MocProfile)]),
    "moc_sn_last_error": (C.c_char_p, [C.c_void_p]),
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


class SNSolver:
    """One DFEM-SN context for a planar box problem; flux and source tensors are device
    FP64 [T, G, 3] (triangle, group, modal coefficient of 1, (x - x_c)/L, (y - y_c)/L).
    n_azim / n_polar default to the problem's."""

    def __init__(self, prob, precision: str = "f32", device: int = 0, max_iter: int = 10000, check_every: int = 1,
                 n_threads: int = 0, n_azim: int | None = None, n_polar: int | None = None):
        L = lib()
        keep = []

        def k(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        xy, tri, tr, rm = k(prob.xy, np.float64), k(prob.tri, np.int32), k(prob.tri_region, np.int32), \
            k(prob.region_material, np.int32)
        m = MocMesh()
        m.n_vertices, m.xy = len(xy), _ptr(xy, _f64)
        m.n_triangles, m.tri, m.tri_region = len(tri), _ptr(tri, _i32), _ptr(tr, _i32)
        m.n_regions, m.region_material = int(prob.n_regions), _ptr(rm, _i32)
        m.domain = int(prob.domain)
        for i in range(4):
            m.box[i] = float(prob.box[i])
        m.hex_apothem = float(prob.hex_apothem)
        for i, b in enumerate(np.asarray(prob.bc).ravel()):
            m.bc[i] = int(b)
        t = MocTracks()
        t.n_azim, t.n_polar, t.spacing = int(n_azim or prob.n_azim), int(n_polar or prob.n_polar), 1.0
        st, ss, nsf, chi = (k(a, np.float64) for a in (prob.sigma_t, prob.sigma_s, prob.nu_sigma_f, prob.chi))
        x = MocXS()
        x.n_materials, x.n_groups = st.shape
        x.sigma_t, x.sigma_s, x.nu_sigma_f, x.chi = _ptr(st, _f64), _ptr(ss, _f64), _ptr(nsf, _f64), _ptr(chi, _f64)
        o = MocOptions(PREC[precision], 0, max_iter, device, check_every, n_threads, 0.0, 0, 0, 0, 0, 0)
        h = C.c_void_p()
        rc = L.moc_sn_create(C.byref(m), C.byref(t), C.byref(x), C.byref(o), C.byref(h))
        if rc != MOC_OK:
            raise MocError(rc, L.moc_sn_last_error(None).decode())
        self._h = h
        self.device = device
        self._refresh_info()
        self.T, self.G = int(len(tri)), int(st.shape[1])

    def close(self):
        if getattr(self, "_h", None) is not None and moc is not None and moc._lib is not None:
            moc._lib.moc_sn_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, ok=(MOC_OK,)):
        if rc not in ok:
            raise MocError(rc, lib().moc_sn_last_error(self._h).decode())
        return rc

    def shape(self):
        return (self.T, self.G, 3)

    def sweep(self, source, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape(), dtype=torch.float64, device=source.device)
        self._check(lib().moc_sn_sweep(self._h, _dptr(source), _dptr(out), _stream_handle(stream)))
        return out

    def solve(self, tol: float = 1e-6, raise_on_noconv: bool = False) -> dict:
        import torch
        torch.cuda.current_stream().synchronize()
        r = MocResult()
        rc = lib().moc_sn_solve(self._h, tol, C.byref(r))
        self._check(rc, (MOC_OK,) if raise_on_noconv else (MOC_OK, MOC_ENOCONV))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk, wall_ms=r.wall_ms,
                    sweeps=r.sweeps, converged=(rc == MOC_OK))

    def run_iterations(self, n: int) -> dict:
        import torch
        torch.cuda.current_stream().synchronize()
        r = MocResult()
        self._check(lib().moc_sn_run_iterations(self._h, int(n), C.byref(r)))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk, wall_ms=r.wall_ms)

    def flux(self, stream=None):
        import torch
        out = torch.empty(self.shape(), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().moc_sn_get_flux(self._h, _dptr(out), _stream_handle(stream)))
        return out

    def set_external_source(self, q):
        import torch
        if q is None:
            self._check(lib().moc_sn_set_external_source(self._h, None))
            return
        torch.cuda.current_stream().synchronize()
        self._check(lib().moc_sn_set_external_source(self._h, _dptr(q.contiguous())))

    def _refresh_info(self):
        inf = MocSnInfo()
        self._check(lib().moc_sn_get_info(self._h, C.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in MocSnInfo._fields_}

    def set_tiles(self, element_tile=None):
        """Sweep tile by tile: element_tile[e] = tile of triangle e (e.g. its pin cell), or
        None for level-by-level sweeps."""
        if element_tile is None:
            self._check(lib().moc_sn_set_tiles(self._h, 0, None))
        else:
            t = np.ascontiguousarray(element_tile, dtype=np.int32)
            if t.shape != (self.T,):
                raise ValueError(f"element_tile must have shape ({self.T},)")
            self._check(lib().moc_sn_set_tiles(self._h, int(t.max()) + 1 if t.size else 0, t.ctypes.data))
        self._refresh_info()

    def set_profiling(self, enable: bool = True):
        self._check(lib().moc_sn_set_profiling(self._h, int(enable)))

    def profile(self) -> dict:
        p = MocProfile()
        self._check(lib().moc_sn_get_profile(self._h, C.byref(p)))
        return dict(sweeps=p.sweeps, sweep_ms=p.sweep_ms, sweep_ms_min=p.sweep_ms_min, sweep_ms_max=p.sweep_ms_max)
