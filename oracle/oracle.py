"""ctypes wrapper around the plain-C FP64 oracle (``moc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package. Arguments are plain numpy
arrays (the problem generators' output), so this module imports nothing from the
product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "moc_oracle.c")


def build(force: bool = False, native: bool = False, out: str | None = None) -> str:
    """Compile the oracle with gcc: plain C11, -O3, OpenMP for the track loop, no
    fast-math. ``native`` adds -march=native for timing on the machine that runs it (the
    default build is portable, since the library may run on another host than the one
    that built it); ``out`` names the library file (default: liboracle.so here)."""
    so = out or _SO
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        tmp = so + ".tmp"
        flags = ["-O3", "-std=c11", "-Wall", "-fPIC", "-shared", "-fopenmp"]
        if native:
            flags.append("-march=native")
        subprocess.check_call(["gcc"] + flags + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, so)
    return so



def build_sanitized(out: str) -> str:
    """The same source built for a sanitizer run (tests only): AddressSanitizer and
    UndefinedBehaviorSanitizer, the process preloading gcc's libasan."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", out, _SRC, "-lm"])
    return out


_lib = None


def lib(path: str | None = None):
    """The oracle library (built here on first use); ``path`` loads another build of the
    same source instead (the benchmark's -march=native copy), before any other use."""
    global _lib
    if _lib is None:
        if path is None:
            build()
        L = C.CDLL(path or _SO)
        P = C.POINTER
        d, i, i64 = C.c_double, C.c_int, C.c_int64
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [i, P(d), i, P(i), P(i), i, P(i), i, P(d), d, P(i), i, i,
                                 P(d), P(d), P(d), P(d), i, i, d, C.c_char_p, i]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_info.argtypes = [C.c_void_p, P(i64), P(d)]
        L.orc_angles.argtypes = [C.c_void_p, P(d), P(d), P(d), P(i), P(i)]
        L.orc_polar.argtypes = [C.c_void_p, P(d), P(d)]
        L.orc_polar_gl.argtypes = [i, P(d), P(d)]
        L.orc_layout.argtypes = [d, d, i, d, P(d), P(d), P(i), P(i), P(d)]
        L.orc_tracks.argtypes = [C.c_void_p, P(i), P(d), P(d), P(i64), P(i)]
        L.orc_segments.argtypes = [C.c_void_p, P(i), P(d)]
        L.orc_volumes.argtypes = [C.c_void_p, P(d)]
        L.orc_get_psi.argtypes = [C.c_void_p, P(d)]
        L.orc_set_psi.argtypes = [C.c_void_p, P(d)]
        L.orc_get_exit_psi.argtypes = [C.c_void_p, P(d)]
        L.orc_set_options.argtypes = [C.c_void_p, i, i]
        L.orc_set_threads.restype = i
        L.orc_set_default_threads.argtypes = [i]
        L.orc_set_threads.argtypes = [C.c_void_p, i]
        L.orc_set_external_source.argtypes = [C.c_void_p, P(d)]
        L.orc_sweep.argtypes = [C.c_void_p, P(d), P(d), P(d)]
        L.orc_set_coarse.restype = i
        L.orc_set_coarse.argtypes = [C.c_void_p, i, P(i)]
        L.orc_coarse_slots.restype = i64
        L.orc_coarse_slots.argtypes = [C.c_void_p]
        L.orc_coarse_adjacency.argtypes = [C.c_void_p, P(i64), P(i)]
        L.orc_currents.argtypes = [C.c_void_p, P(d), P(d)]
        L.orc_solve.restype = i
        L.orc_solve.argtypes = [C.c_void_p, d, i, P(d), P(d), P(i), P(d), P(d), i]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def polar_gl(P: int):
    mu, w = np.zeros(P), np.zeros(P)
    lib().orc_polar_gl(P, _p(mu, C.c_double), _p(w, C.c_double))
    return mu, w


def layout(W: float, H: float, A: int, spacing: float):
    NA = A // 2
    phi, dlt, wa = np.zeros(NA), np.zeros(NA), np.zeros(NA)
    nx, ny = np.zeros(NA, np.int32), np.zeros(NA, np.int32)
    rc = lib().orc_layout(W, H, A, spacing, _p(phi, C.c_double), _p(dlt, C.c_double),
                          _p(nx, C.c_int), _p(ny, C.c_int), _p(wa, C.c_double))
    if rc:
        raise ValueError("n_azim must be a positive multiple of 4")
    return phi, dlt, nx, ny, wa


class Oracle:
    """FP64 reference solver for one problem (mesh + XS + tracking parameters).

    ``xs`` arrays follow the generators' convention: sigma_t [M, G], sigma_s [M, G, G]
    (from, to), nu_sigma_f [M, G], chi [M, G].
    """

    def __init__(self, xy, tri, tri_region, n_regions, region_material, domain, box,
                 hex_apothem, bc, sigma_t, sigma_s, nu_sigma_f, chi, n_azim, n_polar, spacing,
                 threads: int = 1):
        L = lib()
        L.orc_set_default_threads(int(threads))   # tracking and sweeps of this context
        self._keep = [_f64(xy), _i32(tri), _i32(tri_region), _i32(region_material),
                      _f64(box), _i32(bc), _f64(sigma_t), _f64(sigma_s), _f64(nu_sigma_f),
                      _f64(chi)]
        xy, tri, tr, rm, box, bc, st, ss, nsf, chi = self._keep
        self.R = int(n_regions)
        self.M, self.G = st.shape
        self.P = int(n_polar)
        err = C.create_string_buffer(256)
        h = L.orc_create(len(xy), _p(xy, C.c_double), len(tri), _p(tri, C.c_int),
                         _p(tr, C.c_int), self.R, _p(rm, C.c_int), int(domain),
                         _p(box, C.c_double), float(hex_apothem), _p(bc, C.c_int),
                         self.M, self.G, _p(st, C.c_double), _p(ss, C.c_double),
                         _p(nsf, C.c_double), _p(chi, C.c_double), int(n_azim), self.P,
                         float(spacing), err, 256)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self._h = C.c_void_p(h)
        info = np.zeros(4, np.int64)
        gap = C.c_double()
        L.orc_info(self._h, _p(info, C.c_int64), C.byref(gap))
        self.T, self.S, self.NA = int(info[0]), int(info[1]), int(info[2])
        self.max_gap = gap.value
        self.sigma_t = st
        self.region_material = rm

    @classmethod
    def from_problem(cls, p, threads: int = 1):
        return cls(p.xy, p.tri, p.tri_region, p.n_regions, p.region_material, p.domain,
                   p.box, p.hex_apothem, p.bc, p.sigma_t, p.sigma_s, p.nu_sigma_f, p.chi,
                   p.n_azim, p.n_polar, p.spacing, threads=threads)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # --- geometry ------------------------------------------------------------------
    def angles(self):
        n = self.NA
        phi, dlt, wa = np.zeros(n), np.zeros(n), np.zeros(n)
        nx, ny = np.zeros(n, np.int32), np.zeros(n, np.int32)
        lib().orc_angles(self._h, _p(phi, C.c_double), _p(dlt, C.c_double), _p(wa, C.c_double),
                         _p(nx, C.c_int), _p(ny, C.c_int))
        return dict(phi=phi, delta=dlt, w=wa, nx=nx, ny=ny)

    def polar(self):
        mu, w = np.zeros(self.P), np.zeros(self.P)
        lib().orc_polar(self._h, _p(mu, C.c_double), _p(w, C.c_double))
        return mu, w

    def tracks(self):
        T = self.T
        ang = np.zeros(T, np.int32)
        xy = np.zeros((T, 4))
        ln = np.zeros(T)
        off = np.zeros(T + 1, np.int64)
        link = np.zeros((T, 2), np.int32)
        lib().orc_tracks(self._h, _p(ang, C.c_int), _p(xy, C.c_double), _p(ln, C.c_double),
                         _p(off, C.c_int64), _p(link, C.c_int))
        return dict(angle=ang, xy=xy, length=ln, offset=off, link=link)

    def segments(self):
        reg = np.zeros(self.S, np.int32)
        ln = np.zeros(self.S)
        lib().orc_segments(self._h, _p(reg, C.c_int), _p(ln, C.c_double))
        return reg, ln

    def volumes(self):
        V = np.zeros(self.R)
        lib().orc_volumes(self._h, _p(V, C.c_double))
        return V

    # --- state ---------------------------------------------------------------------
    def psi_shape(self):
        return (self.T, 2, self.P, self.G)

    def get_psi(self):
        a = np.zeros(self.psi_shape())
        lib().orc_get_psi(self._h, _p(a, C.c_double))
        return a

    def set_psi(self, psi):
        a = _f64(np.broadcast_to(psi, self.psi_shape()))
        lib().orc_set_psi(self._h, _p(a, C.c_double))

    def get_exit_psi(self):
        a = np.zeros(self.psi_shape())
        lib().orc_get_exit_psi(self._h, _p(a, C.c_double))
        return a

    def set_options(self, gs_boundary=False, gs_energy=False):
        lib().orc_set_options(self._h, int(gs_boundary), int(gs_energy))

    def set_threads(self, n: int) -> bool:
        """Threads of the sweep's track loop (1 = serial, the default). Returns whether the
        library was built with OpenMP."""
        return bool(lib().orc_set_threads(self._h, int(n)))

    def set_external_source(self, q):
        if q is None:
            lib().orc_set_external_source(self._h, None)
        else:
            self._qext = _f64(q).reshape(self.R, self.G)
            lib().orc_set_external_source(self._h, _p(self._qext, C.c_double))

    # --- coarse mesh (CMFD currents) ---------------------------------------------------
    def set_coarse(self, n_cells, region_cell):
        """Assign every region to a coarse cell; later sweeps tally the partial currents
        across the coarse-cell surfaces that the tracks cross."""
        self._cell = _i32(region_cell)
        self.n_cells = int(n_cells)
        if lib().orc_set_coarse(self._h, self.n_cells, _p(self._cell, C.c_int)):
            raise ValueError("oracle: region_cell out of range")

    def coarse_adjacency(self):
        """(off [C+1], nbr [slots]): the neighbour cells of each cell, -1 = boundary."""
        n = int(lib().orc_coarse_slots(self._h))
        off = np.zeros(self.n_cells + 1, np.int64)
        nbr = np.zeros(max(n, 1), np.int32)
        lib().orc_coarse_adjacency(self._h, _p(off, C.c_int64), _p(nbr, C.c_int))
        return off, nbr[:n]

    def currents(self):
        """Partial currents of the last sweep: jpart [slots, G] leaving each cell through
        each slot, jin [C, G] entering each cell from outside the domain."""
        n = int(lib().orc_coarse_slots(self._h))
        jp = np.zeros((max(n, 1), self.G))
        jin = np.zeros((self.n_cells, self.G))
        lib().orc_currents(self._h, _p(jp, C.c_double), _p(jin, C.c_double))
        return jp[:n], jin

    # --- compute -------------------------------------------------------------------
    def sweep(self, src, return_tally=False):
        """One sweep for an emission density src [R, G]; returns phi [R, G]."""
        s = _f64(src).reshape(self.R, self.G)
        phi = np.zeros((self.R, self.G))
        T = np.zeros((self.R, self.G)) if return_tally else None
        lib().orc_sweep(self._h, _p(s, C.c_double), _p(phi, C.c_double),
                        _p(T, C.c_double) if T is not None else None)
        return (phi, T) if return_tally else phi

    def solve(self, tol=1e-6, max_iter=10000, phi0=None, k0=1.0, eigen=True):
        phi = np.ones((self.R, self.G)) if phi0 is None else _f64(phi0).reshape(self.R, self.G).copy()
        k = C.c_double(k0)
        it = C.c_int()
        res, dk = C.c_double(), C.c_double()
        rc = lib().orc_solve(self._h, tol, max_iter, _p(phi, C.c_double), C.byref(k),
                             C.byref(it), C.byref(res), C.byref(dk), int(eigen))
        return dict(phi=phi, k=k.value, iterations=it.value, residual=res.value, dk=dk.value,
                    converged=(rc == 0))
