"""Python binding of libmoc (include/moc.h): argument marshalling only.

Every step of the transport path runs in libmoc's C++ host setup and HIP kernels; this
module converts numpy arrays and torch device tensors into the C structures and
pointers the ABI takes. PyTorch is used only to own device memory and streams.

If ``libmoc.so`` has not been built the import of :func:`lib` raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmoc.so")

MOC_OK, MOC_EINVAL, MOC_ENOMEM, MOC_EHIP, MOC_ENOCONV, MOC_ESTATE = range(6)
PREC = {"f32": 0, "f64": 1}
EXP = {"poly": 0, "table": 1, "libm": 2, "diff": 3}
FLAG_FELL_BACK_TO_COLD = 1
FLAG_FIXED_SOURCE = 2

_i32, _i64, _f64 = C.c_int32, C.c_int64, C.c_double
_P = C.POINTER


class MocMesh(C.Structure):
    _fields_ = [("n_vertices", _i32), ("xy", _P(_f64)), ("n_triangles", _i32), ("tri", _P(_i32)),
                ("tri_region", _P(_i32)), ("n_regions", _i32), ("region_material", _P(_i32)),
                ("domain", _i32), ("box", _f64 * 4), ("hex_apothem", _f64), ("bc", _i32 * 6)]


class MocTracks(C.Structure):
    _fields_ = [("n_azim", _i32), ("n_polar", _i32), ("spacing", _f64),
                ("polar_mu", _P(_f64)), ("polar_w", _P(_f64))]


class MocXS(C.Structure):
    _fields_ = [("n_materials", _i32), ("n_groups", _i32), ("sigma_t", _P(_f64)),
                ("sigma_s", _P(_f64)), ("nu_sigma_f", _P(_f64)), ("chi", _P(_f64))]


class MocOptions(C.Structure):
    _fields_ = [("precision", _i32), ("exp_mode", _i32), ("max_iter", _i32), ("device", _i32),
                ("check_every", _i32), ("n_threads", _i32), ("window_cm", _f64),
                ("tally_slots", _i32), ("group_batch", _i32), ("window_steps", _i32),
                ("lane_stagger", _i32), ("batch_order", _i32)]


class MocResult(C.Structure):
    _fields_ = [("k", _f64), ("iterations", _i32), ("residual", _f64), ("dk", _f64),
                ("wall_ms", _f64), ("flags", _i32), ("sweeps", _i32)]


class MocInfo(C.Structure):
    _fields_ = [("n_regions", _i32), ("n_groups", _i32), ("n_materials", _i32), ("n_polar", _i32),
                ("n_angles", _i32), ("n_tracks", _i32), ("n_segments", _i64), ("n_updates", _i64),
                ("n_padded_steps", _i64), ("n_batches", _i32), ("n_windows", _i64),
                ("n_window_slots", _i64), ("window_cm", _f64), ("max_window_slots", _i32),
                ("setup_ms", _f64),
                ("device_bytes", _i64), ("precision", _i32), ("lane_stagger", _i32)]


class MocProfile(C.Structure):
    _fields_ = [("sweeps", _i64), ("sweep_ms", _f64), ("sweep_ms_min", _f64), ("sweep_ms_max", _f64),
                ("cmfd_steps", _i64), ("cmfd_ms", _f64)]


class MocCmfdOptions(C.Structure):
    _fields_ = [("tol", _f64), ("shift", _f64), ("max_outer", _i32), ("max_inner", _i32),
                ("coarse_blocks", _i32)]


class MocCoarseInfo(C.Structure):
    _fields_ = [("n_cells", _i32), ("n_surfaces", _i32), ("n_crossings", _i64), ("setup_ms", _f64),
                ("last_outer", _i32), ("last_inner", _i32), ("last_k", _f64)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "moc_create": (C.c_int, [_P(MocMesh), _P(MocTracks), _P(MocXS), _P(MocOptions), _P(C.c_void_p)]),
    "moc_destroy": (None, [C.c_void_p]),
    "moc_sweep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_solve": (C.c_int, [C.c_void_p, _f64, _P(MocResult)]),
    "moc_run_iterations": (C.c_int, [C.c_void_p, C.c_int, _P(MocResult)]),
    "moc_set_initial_guess": (C.c_int, [C.c_void_p, C.c_void_p, _f64, C.c_void_p]),
    "moc_get_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_get_boundary_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_set_boundary_flux": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "moc_set_exit_flux_buffer": (C.c_int, [C.c_void_p, C.c_void_p]),
    "moc_set_external_source": (C.c_int, [C.c_void_p, C.c_void_p]),
    "moc_get_info": (C.c_int, [C.c_void_p, _P(MocInfo)]),
    "moc_get_volumes": (C.c_int, [C.c_void_p, _P(_f64)]),
    "moc_get_tracks": (C.c_int, [C.c_void_p, _P(_i32), _P(_f64), _P(_i64), _P(_i32), _P(_f64), _P(_i32)]),
    "moc_get_packing": (C.c_int, [C.c_void_p, _P(_i64), _P(_i32), _P(_i64), _P(_i32), _P(_i64),
                                 _P(_i32), _P(_i32), _P(_f64), _P(C.c_uint32), _P(_i32)]),
    "moc_get_quadrature": (C.c_int, [C.c_void_p, _P(_f64), _P(_f64), _P(_f64), _P(_f64), _P(_f64)]),
    "moc_last_error": (C.c_char_p, [C.c_void_p]),
    "moc_set_profiling": (C.c_int, [C.c_void_p, C.c_int]),
    "moc_set_materials": (C.c_int, [C.c_void_p, _P(_i32), _P(MocXS)]),
    "moc_locate_points": (C.c_int, [C.c_void_p, _P(_f64), _i64, _P(_i32)]),
    "moc_get_centroids": (C.c_int, [C.c_void_p, _P(_f64)]),
    "moc_get_profile": (C.c_int, [C.c_void_p, _P(MocProfile)]),
    "moc_set_coarse_mesh": (C.c_int, [C.c_void_p, _i32, _P(_i32), _P(MocCmfdOptions)]),
    "moc_get_coarse_info": (C.c_int, [C.c_void_p, _P(MocCoarseInfo)]),
    "moc_get_surface_currents": (C.c_int, [C.c_void_p, _P(_i32), _P(_f64)]),
}

_lib = None


def lib():
    """Load libmoc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_01591_amd.build`")
        # torch first: its wheel carries its own HIP runtime under the same soname as the
        # system one libmoc links, and the first one loaded serves the whole process. Loaded
        # the other way round, torch runs on a runtime it was not built with and finds no GPU.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmoc error {code}: {msg}")
        self.code = code


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(_P(ct))


def _dptr(t) -> int:
    """Device pointer of a contiguous torch CUDA tensor."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Solver:
    """One libmoc context for a problem (see ``problems.Problem``).

    precision: "f32" (FP32 sweep, FP64 source/eigenvalue/norms/tallies) or "f64".
    device: HIP device ordinal, or -1 for a host-only context (tracking, volumes,
    quadrature and info; no sweeps).
    """

    def __init__(self, prob, precision: str = "f32", exp_mode: str = "poly", device: int = 0,
                 max_iter: int = 10000, check_every: int = 1, n_threads: int = 0,
                 polar: Optional[tuple] = None, window_cm: float = 0.0, tally_slots: int = 0,
                 group_batch: int = 0, window_steps: int = 0, lane_stagger: int = 0, batch_order: int = 0):
        L = lib()
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        xy = keep(prob.xy, np.float64)
        tri = keep(prob.tri, np.int32)
        tr = keep(prob.tri_region, np.int32)
        rm = keep(prob.region_material, np.int32)
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
        t.n_azim, t.n_polar, t.spacing = int(prob.n_azim), int(prob.n_polar), float(prob.spacing)
        if polar is not None:
            mu, w = keep(polar[0], np.float64), keep(polar[1], np.float64)
            t.polar_mu, t.polar_w = _ptr(mu, _f64), _ptr(w, _f64)
        st = keep(prob.sigma_t, np.float64)
        ss = keep(prob.sigma_s, np.float64)
        nsf = keep(prob.nu_sigma_f, np.float64)
        chi = keep(prob.chi, np.float64)
        x = MocXS()
        x.n_materials, x.n_groups = st.shape
        x.sigma_t, x.sigma_s, x.nu_sigma_f, x.chi = (_ptr(st, _f64), _ptr(ss, _f64),
                                                     _ptr(nsf, _f64), _ptr(chi, _f64))
        o = MocOptions(PREC[precision], EXP[exp_mode], max_iter, device, check_every, n_threads,
                       float(window_cm), int(tally_slots), int(group_batch), int(window_steps),
                       int(lane_stagger), int(batch_order))
        h = C.c_void_p()
        rc = L.moc_create(C.byref(m), C.byref(t), C.byref(x), C.byref(o), C.byref(h))
        if rc != MOC_OK:
            raise MocError(rc, L.moc_last_error(None).decode())
        self._h = h
        self._keep = []
        self.device = device
        self.precision = precision
        self._refresh_info()
        inf = self.info
        self.R, self.G, self.P = inf["n_regions"], inf["n_groups"], inf["n_polar"]
        self.T, self.S, self.U = inf["n_tracks"], inf["n_segments"], inf["n_updates"]
        self._exit = None
        self._qext = None

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.moc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, ok=(MOC_OK,)):
        if rc not in ok:
            raise MocError(rc, lib().moc_last_error(self._h).decode())
        return rc

    # ---------------------------------------------------------------- device calls
    def sweep(self, source, out=None, stream=None):
        """One sweep for an emission density ``source`` (device FP64 [R, G]); returns
        the scalar flux (device FP64 [R, G]). Enqueued on the current torch stream."""
        import torch
        if out is None:
            out = torch.empty((self.R, self.G), dtype=torch.float64, device=source.device)
        self._check(lib().moc_sweep(self._h, _dptr(source), _dptr(out), _stream_handle(stream)))
        return out

    def solve(self, tol: float = 1e-6, raise_on_noconv: bool = False) -> dict:
        import torch
        torch.cuda.current_stream().synchronize()
        r = MocResult()
        rc = lib().moc_solve(self._h, tol, C.byref(r))
        self._check(rc, (MOC_OK,) if raise_on_noconv else (MOC_OK, MOC_ENOCONV))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk,
                    wall_ms=r.wall_ms, flags=r.flags, sweeps=r.sweeps, converged=(rc == MOC_OK))

    def flux(self, stream=None):
        import torch
        out = torch.empty((self.R, self.G), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().moc_get_flux(self._h, _dptr(out), _stream_handle(stream)))
        return out

    def psi_shape(self):
        return (self.T, 2, self.P, self.G)

    def get_boundary_flux(self, stream=None):
        import torch
        out = torch.empty(self.psi_shape(), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().moc_get_boundary_flux(self._h, _dptr(out), _stream_handle(stream)))
        return out

    def set_boundary_flux(self, psi, stream=None):
        self._keep_psi = psi.contiguous()
        self._check(lib().moc_set_boundary_flux(self._h, _dptr(self._keep_psi), _stream_handle(stream)))

    def set_exit_buffer(self, buf):
        """Record the outgoing angular flux of every track-sense in ``buf`` (device FP64
        [T, 2, P, G]) on every following sweep; None disables."""
        self._exit = buf
        self._check(lib().moc_set_exit_flux_buffer(self._h, None if buf is None else _dptr(buf)))

    def set_external_source(self, q):
        import torch
        if q is None:
            self._check(lib().moc_set_external_source(self._h, None))
            return
        torch.cuda.current_stream().synchronize()
        self._check(lib().moc_set_external_source(self._h, _dptr(q.contiguous())))

    def set_initial_guess(self, phi0, k0: float = 1.0, psi0=None):
        import torch
        torch.cuda.current_stream().synchronize()
        self._check(lib().moc_set_initial_guess(self._h, _dptr(phi0), float(k0),
                                                None if psi0 is None else _dptr(psi0)))

    def set_profiling(self, enable: bool = True):
        self._check(lib().moc_set_profiling(self._h, int(enable)))

    def profile(self) -> dict:
        p = MocProfile()
        self._check(lib().moc_get_profile(self._h, C.byref(p)))
        return dict(sweeps=p.sweeps, sweep_ms=p.sweep_ms, sweep_ms_min=p.sweep_ms_min,
                    sweep_ms_max=p.sweep_ms_max, cmfd_steps=p.cmfd_steps, cmfd_ms=p.cmfd_ms)

    def run_iterations(self, n: int) -> dict:
        """Exactly n power (or source) iterations from a cold start, with one
        convergence read-back at the end (used for timing)."""
        r = MocResult()
        import torch
        torch.cuda.current_stream().synchronize()
        self._check(lib().moc_run_iterations(self._h, int(n), C.byref(r)))
        return dict(k=r.k, iterations=r.iterations, residual=r.residual, dk=r.dk, wall_ms=r.wall_ms,
                    flags=r.flags, sweeps=r.sweeps)

    def set_materials(self, prob):
        """Swap in the cross sections and material map of ``prob`` (same mesh)."""
        rm = np.ascontiguousarray(prob.region_material, np.int32)
        arrs = [np.ascontiguousarray(a, np.float64) for a in (prob.sigma_t, prob.sigma_s, prob.nu_sigma_f, prob.chi)]
        x = MocXS()
        x.n_materials, x.n_groups = arrs[0].shape
        x.sigma_t, x.sigma_s, x.nu_sigma_f, x.chi = (_ptr(a, _f64) for a in arrs)
        self._check(lib().moc_set_materials(self._h, _ptr(rm, _i32), C.byref(x)))

    def _refresh_info(self):
        inf = MocInfo()
        lib().moc_get_info(self._h, C.byref(inf))
        self.info = {k: getattr(inf, k) for k, _ in MocInfo._fields_}

    def set_coarse_mesh(self, n_cells: int, region_cell=None, tol: float = 0.0, shift: float = 0.0,
                        max_outer: int = 0, max_inner: int = 0, coarse_blocks: int = 0):
        """CMFD on a coarse mesh: region_cell [R] (user order) assigns regions to cells;
        n_cells = 0 removes it. Zero options take the library defaults."""
        o = MocCmfdOptions(float(tol), float(shift), int(max_outer), int(max_inner), int(coarse_blocks))
        if n_cells <= 0 or region_cell is None:
            self._check(lib().moc_set_coarse_mesh(self._h, 0, None, C.byref(o)))
        else:
            rc = np.ascontiguousarray(region_cell, np.int32)
            if rc.shape != (self.R,):
                raise ValueError("region_cell must have one entry per region")
            self._check(lib().moc_set_coarse_mesh(self._h, int(n_cells), _ptr(rc, _i32), C.byref(o)))
        self._refresh_info()

    def coarse_info(self) -> dict:
        ci = MocCoarseInfo()
        self._check(lib().moc_get_coarse_info(self._h, C.byref(ci)))
        return {k: getattr(ci, k) for k, _ in MocCoarseInfo._fields_}

    def surface_currents(self, with_current: bool = True):
        """(cells [Ns, 2], current [Ns, G] or None): net currents of the last sweep."""
        ns = self.coarse_info()["n_surfaces"]
        cells = np.zeros((ns, 2), np.int32)
        cur = np.zeros((ns, self.G)) if with_current else None
        self._check(lib().moc_get_surface_currents(self._h, _ptr(cells, _i32),
                                                   _ptr(cur, _f64) if cur is not None else None))
        return cells, cur

    def locate(self, xy) -> np.ndarray:
        xy = np.ascontiguousarray(xy, np.float64).reshape(-1, 2)
        out = np.zeros(len(xy), np.int32)
        self._check(lib().moc_locate_points(self._h, _ptr(xy, _f64), len(xy), _ptr(out, _i32)))
        return out

    def centroids(self) -> np.ndarray:
        out = np.zeros((self.R, 2))
        self._check(lib().moc_get_centroids(self._h, _ptr(out, _f64)))
        return out

    # ---------------------------------------------------------------- host queries
    def volumes(self) -> np.ndarray:
        V = np.zeros(self.R)
        self._check(lib().moc_get_volumes(self._h, _ptr(V, _f64)))
        return V

    def quadrature(self) -> dict:
        NA, P = self.info["n_angles"], self.P
        phi, dl, wa = np.zeros(NA), np.zeros(NA), np.zeros(NA)
        mu, wp = np.zeros(P), np.zeros(P)
        self._check(lib().moc_get_quadrature(self._h, _ptr(phi, _f64), _ptr(dl, _f64), _ptr(wa, _f64),
                                             _ptr(mu, _f64), _ptr(wp, _f64)))
        return dict(phi=phi, delta=dl, w=wa, mu=mu, w_polar=wp)

    def packing(self) -> dict:
        """Packed sweep layout (host-only contexts)."""
        nb, nw, ns = self.info["n_batches"], self.info["n_windows"], self.info["n_window_slots"]
        ne = self.info["n_padded_steps"]
        out = dict(batch_win=np.zeros(nb + 1, np.int64), batch_angle=np.zeros(nb, np.int32),
                   win_entry_off=np.zeros(nw, np.int64), win_nsteps=np.zeros(nw, np.int32),
                   win_tab_off=np.zeros(nw, np.int64), win_nslots=np.zeros(nw, np.int32),
                   win_tab=np.zeros(ns, np.int32), seg_len=np.zeros(ne), seg_key=np.zeros(ne, np.uint32),
                   user_of_internal=np.zeros(self.R, np.int32))
        self._check(lib().moc_get_packing(
            self._h, _ptr(out["batch_win"], _i64), _ptr(out["batch_angle"], _i32),
            _ptr(out["win_entry_off"], _i64), _ptr(out["win_nsteps"], _i32),
            _ptr(out["win_tab_off"], _i64), _ptr(out["win_nslots"], _i32), _ptr(out["win_tab"], _i32),
            _ptr(out["seg_len"], _f64), _ptr(out["seg_key"], C.c_uint32),
            _ptr(out["user_of_internal"], _i32)))
        return out

    def tracks_angles(self) -> np.ndarray:
        """Track angle index of every canonical track (no segment dump)."""
        ang = np.zeros(self.T, np.int32)
        self._check(lib().moc_get_tracks(self._h, _ptr(ang, _i32), None, None, None, None, None))
        return ang

    def tracks(self) -> dict:
        T, S = self.T, self.S
        ang = np.zeros(T, np.int32)
        xy = np.zeros((T, 4))
        off = np.zeros(T + 1, np.int64)
        reg = np.zeros(S, np.int32)
        ln = np.zeros(S)
        link = np.zeros((T, 2), np.int32)
        self._check(lib().moc_get_tracks(self._h, _ptr(ang, _i32), _ptr(xy, _f64), _ptr(off, _i64),
                                         _ptr(reg, _i32), _ptr(ln, _f64), _ptr(link, _i32)))
        return dict(angle=ang, xy=xy, offset=off, region=reg, length=ln, link=link)
