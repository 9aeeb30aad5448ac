"""Seeded synthetic problem generators: triangular meshes and multigroup cross sections.

This module produces *inputs* only (geometry, material maps, cross sections, tracking
parameters). It holds none of the transport method's arithmetic, so both the HIP path
and the FP64 oracle can consume what it writes without sharing any solver code.

The workloads stand in for the paper's benchmark problems (C5G7-like square pin
lattices with 7 groups, Sec. 4.1; ABTR/Empire-like hexagonal lattices with a fast
group structure, Sec. 4.2), whose cross sections and meshes are not available. Every
draw uses ``numpy.random.default_rng`` (PCG64) in a fixed order, documented on each
function.

Cross-section convention: ``sigma_s[m, gp, g]`` is the transfer from group ``gp`` to
group ``g`` (isotropic, Eq. MGNTE restricted to the L = 0 term).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BC_VACUUM = 0
BC_REFLECTIVE = 1
DOMAIN_BOX = 0
DOMAIN_HEXAGON = 1


@dataclasses.dataclass
class Problem:
    """A complete planar transport problem.

    Arrays are C-contiguous. ``bc`` holds one code per domain side: for a box the
    order is (x = x0, x = x1, y = y0, y = y1); a hexagon has six sides, all with the
    same code here.
    """
    name: str
    xy: np.ndarray            # float64 [Nv, 2]
    tri: np.ndarray           # int32 [Nt, 3], counter-clockwise
    tri_region: np.ndarray    # int32 [Nt]
    n_regions: int
    region_material: np.ndarray  # int32 [R]
    domain: int               # DOMAIN_BOX | DOMAIN_HEXAGON
    box: tuple                # (x0, y0, x1, y1) bounding box of the domain
    hex_apothem: float        # hexagon only: centre-to-flat distance (flats parallel to x)
    bc: np.ndarray            # int32 [4] (box) or [6] (hexagon)
    sigma_t: np.ndarray       # float64 [M, G]
    sigma_s: np.ndarray       # float64 [M, G, G]  (from gp, to g)
    nu_sigma_f: np.ndarray    # float64 [M, G]
    chi: np.ndarray           # float64 [M, G]
    n_azim: int
    n_polar: int
    spacing: float

    @property
    def n_groups(self) -> int:
        return int(self.sigma_t.shape[1])

    @property
    def n_materials(self) -> int:
        return int(self.sigma_t.shape[0])

    def region_areas(self) -> np.ndarray:
        """Exact polygon areas of the regions (sum of their triangles)."""
        a = tri_areas(self.xy, self.tri)
        out = np.zeros(self.n_regions)
        np.add.at(out, self.tri_region, a)
        return out

    def with_xs(self, sigma_t, sigma_s, nu_sigma_f, chi, region_material=None) -> "Problem":
        p = dataclasses.replace(self)
        p.sigma_t = np.ascontiguousarray(sigma_t, dtype=np.float64)
        p.sigma_s = np.ascontiguousarray(sigma_s, dtype=np.float64)
        p.nu_sigma_f = np.ascontiguousarray(nu_sigma_f, dtype=np.float64)
        p.chi = np.ascontiguousarray(chi, dtype=np.float64)
        if region_material is not None:
            p.region_material = np.ascontiguousarray(region_material, dtype=np.int32)
        return p


# ----------------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------------

def tri_areas(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1])
                  - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))


def _dedup(xy: np.ndarray, tri: np.ndarray, quantum: float = 1e-8):
    key = np.round(xy / quantum).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    return np.ascontiguousarray(xy[first]), inv[tri].astype(np.int32)


def _min_incident_edge(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    h = np.full(len(xy), np.inf)
    for e0, e1 in ((0, 1), (1, 2), (2, 0)):
        u, v = tri[:, e0], tri[:, e1]
        L = np.hypot(*(xy[u] - xy[v]).T)
        np.minimum.at(h, u, L)
        np.minimum.at(h, v, L)
    return h


def _jitter(xy, tri, movable, rng, frac=0.10):
    """Move each movable vertex by U[-frac*h, frac*h]^2 (h = shortest incident edge),
    then undo moves that invert a triangle until every triangle is positive."""
    h = _min_incident_edge(xy, tri)
    d = rng.uniform(-frac, frac, size=xy.shape) * h[:, None]
    d[~movable] = 0.0
    new = xy + d
    for _ in range(20):
        bad = tri_areas(new, tri) <= 1e-14
        if not bad.any():
            break
        vb = np.unique(tri[bad].reshape(-1))
        new[vb] = xy[vb]
    assert (tri_areas(new, tri) > 0).all()
    return new


def _ring_tris(inner: np.ndarray, outer: np.ndarray, flips: np.ndarray) -> np.ndarray:
    """Triangulate the band between two closed vertex loops with equal counts.
    ``inner``/``outer`` are index arrays in counter-clockwise order."""
    n = len(inner)
    j = np.arange(n)
    jn = (j + 1) % n
    i0, i1, o0, o1 = inner[j], inner[jn], outer[j], outer[jn]
    a = np.where(flips[:, None], np.stack([i0, o0, i1], 1), np.stack([i0, o0, o1], 1))
    b = np.where(flips[:, None], np.stack([o0, o1, i1], 1), np.stack([i0, o1, i1], 1))
    return np.concatenate([a, b])


# ----------------------------------------------------------------------------------
# square pin template
# ----------------------------------------------------------------------------------

def _square_boundary(pitch: float, m: int) -> np.ndarray:
    """4m points on the square [-p/2, p/2]^2, uniform along each side, counter-clockwise
    starting at the corner (p/2, -p/2)."""
    h = pitch / 2.0
    t = np.arange(m) / m
    right = np.stack([np.full(m, h), -h + 2 * h * t], 1)
    top = np.stack([h - 2 * h * t, np.full(m, h)], 1)
    left = np.stack([np.full(m, -h), h - 2 * h * t], 1)
    bottom = np.stack([-h + 2 * h * t, np.full(m, -h)], 1)
    return np.concatenate([right, top, left, bottom])


def _pin_template(pitch, r_fuel, m, n_fuel_rings, n_mod_rings, rng, boundary=None):
    """One square pin cell: centre fan, fuel rings (equal-area radii, area-preserving
    polygons), moderator rings blending the fuel polygon to the cell boundary.
    Returns (xy, tri, is_fuel)."""
    B = _square_boundary(pitch, m) if boundary is None else boundary
    ns = len(B)
    th = np.arctan2(B[:, 1], B[:, 0])
    dth = np.diff(np.concatenate([th, th[:1] + 2 * np.pi]))
    dth = np.mod(dth, 2 * np.pi)
    kappa = math.sqrt(2 * math.pi / np.sum(np.sin(dth)))
    u = np.stack([np.cos(th), np.sin(th)], 1)
    pts = [np.zeros((1, 2))]
    loops = []
    nxt = 1
    for i in range(1, n_fuel_rings + 1):
        r = r_fuel * math.sqrt(i / n_fuel_rings) * kappa
        pts.append(r * u)
        loops.append(np.arange(nxt, nxt + ns))
        nxt += ns
    C = kappa * r_fuel * u
    for k in range(1, n_mod_rings + 1):
        pts.append(C + (k / n_mod_rings) * (B - C))
        loops.append(np.arange(nxt, nxt + ns))
        nxt += ns
    xy = np.concatenate(pts)
    j = np.arange(ns)
    tris = [np.stack([np.zeros(ns, int), loops[0][j], loops[0][(j + 1) % ns]], 1)]
    fuel = [np.ones(ns, bool)]
    for li in range(1, len(loops)):
        flips = rng.random(ns) < 0.5
        t = _ring_tris(loops[li - 1], loops[li], flips)
        tris.append(t)
        fuel.append(np.full(len(t), li < n_fuel_rings))
    tri = np.concatenate(tris).astype(np.int64)
    is_fuel = np.concatenate(fuel)
    assert (tri_areas(xy, tri) > 0).all()
    return xy, tri, is_fuel


# ----------------------------------------------------------------------------------
# cross sections
# ----------------------------------------------------------------------------------

def draw_xs(rng: np.random.Generator, n_fuel: int, n_other: int, G: int,
            sigt_range=(0.2, 2.0), band: Optional[int] = None, upscatter: bool = True):
    """Synthetic multigroup cross sections.

    Per material (fuel types first, then the non-fissile ones) and per group g, in this
    order: Sigma_t ~ U[sigt_range]; scattering ratio c ~ U[0.3, 0.95] so that the
    out-scatter total is c*Sigma_t; destination weights ~ U(0, 1] over the allowed
    destinations, normalised. Allowed destinations are g..G-1 (lower-triangular
    downscatter plus self) and, if ``upscatter``, the single transfer G-1 -> G-2; with
    ``band`` they are g..min(g+band, G-1). Then, for fuel materials only:
    nu*Sigma_f = U[0.5, 2.0] * Sigma_a per group, and chi from normalised U(0, 1] draws
    over the first max(3, ceil(G/4)) groups (capped at G).
    """
    M = n_fuel + n_other
    st = np.zeros((M, G))
    ss = np.zeros((M, G, G))
    nsf = np.zeros((M, G))
    chi = np.zeros((M, G))
    lo, hi = sigt_range
    for m in range(M):
        for g in range(G):
            st[m, g] = rng.uniform(lo, hi)
            c = rng.uniform(0.3, 0.95)
            if band is None:
                dest = list(range(g, G))
                if upscatter and G >= 2 and g == G - 1:
                    dest = [G - 2, G - 1]
            else:
                dest = list(range(g, min(g + band, G - 1) + 1))
            w = 1.0 - rng.random(len(dest))      # U(0, 1]
            w /= w.sum()
            ss[m, g, dest] = c * st[m, g] * w
        if m < n_fuel:
            sa = st[m] - ss[m].sum(axis=1)
            nsf[m] = rng.uniform(0.5, 2.0, size=G) * sa
            nchi = min(G, max(3, math.ceil(G / 4)))
            w = 1.0 - rng.random(nchi)
            chi[m, :nchi] = w / w.sum()
    return st, ss, nsf, chi


# ----------------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------------

def pin_cell_8region(seed: int = 1, G: int = 7, n_azim: int = 16, n_polar: int = 3,
                     spacing: float = 0.05) -> Problem:
    """Single square pin cell, pitch 1.26 cm, fuel circle r = 0.54 cm, 8 regions with
    D2 symmetry: inner fuel disc (r <= 0.54/sqrt 2) split at y = 0 (regions 0, 1), fuel
    annulus split at y = 0 (2, 3), moderator split into quadrants by x = 0 and y = 0
    (4..7). Circles are area-preserving 64-gons with vertices on the axes. Reflective
    on all sides. Materials: 0 = fuel, 1 = moderator. No jitter (symmetry is kept)."""
    pitch, rf = 1.26, 0.54
    ns = 64
    th = 2 * np.pi * np.arange(ns) / ns
    u = np.stack([np.cos(th), np.sin(th)], 1)
    B = u * (pitch / 2) / np.maximum(np.abs(u[:, 0]), np.abs(u[:, 1]))[:, None]
    kappa = math.sqrt(2 * math.pi / (ns * math.sin(2 * math.pi / ns)))
    r_in = rf / math.sqrt(2)
    pts = [np.zeros((1, 2)), kappa * r_in * u, kappa * rf * u]
    C = kappa * rf * u
    n_mod = 2
    for k in range(1, n_mod + 1):
        pts.append(C + (k / n_mod) * (B - C))
    xy = np.concatenate(pts)
    loops = [1 + i * ns + np.arange(ns) for i in range(2 + n_mod)]
    j = np.arange(ns)
    tris = [np.stack([np.zeros(ns, int), loops[0][j], loops[0][(j + 1) % ns]], 1)]
    for li in range(1, len(loops)):
        tris.append(_ring_tris(loops[li - 1], loops[li], np.zeros(ns, bool)))
    tri = np.concatenate(tris)
    cen = xy[tri].mean(axis=1)
    rc = np.hypot(cen[:, 0], cen[:, 1])
    up = cen[:, 1] > 0
    region = np.empty(len(tri), np.int32)
    disc = rc < kappa * r_in
    ann = (~disc) & (rc < kappa * rf)
    mod = ~(disc | ann)
    region[disc] = np.where(up[disc], 0, 1)
    region[ann] = np.where(up[ann], 2, 3)
    qx, qy = cen[mod, 0] > 0, cen[mod, 1] > 0
    region[mod] = np.where(qy, np.where(qx, 4, 5), np.where(qx, 7, 6))
    xy = xy + pitch / 2           # domain [0, 1.26]^2
    rng = np.random.default_rng(seed)
    st, ss, nsf, chi = draw_xs(rng, 1, 1, G)
    return Problem("cfg1_pincell", np.ascontiguousarray(xy), tri.astype(np.int32), region, 8,
                   np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32), DOMAIN_BOX,
                   (0.0, 0.0, pitch, pitch), 0.0,
                   np.full(4, BC_REFLECTIVE, np.int32), st, ss, nsf, chi,
                   n_azim, n_polar, spacing)


def square_lattice(npx: int, npy: int, *, seed: int, mesh_seed: Optional[int] = None,
                   pitch: float = 1.26, r_fuel: float = 0.54, m: int = 3,
                   n_fuel_rings: int = 2, n_mod_rings: int = 3, G: int = 7,
                   n_fuel_types: int = 3, bc=(1, 1, 1, 1), n_azim: int = 64,
                   n_polar: int = 3, spacing: float = 0.02, jitter: float = 0.10,
                   name: str = "lattice") -> Problem:
    """npx x npy square pin lattice with one triangle per region.

    Draw order. From ``default_rng(seed)``: cross sections for ``n_fuel_types`` fuel
    materials then one moderator (``draw_xs``), then each pin's fuel type (uniform
    integer, row-major pin order). From ``default_rng(mesh_seed)`` (default: seed):
    each pin's quad-split diagonals, the vertex jitter, then the random region
    numbering. Materials are ordered [fuel types..., moderator]."""
    rng = np.random.default_rng(seed)
    mrng = np.random.default_rng(seed if mesh_seed is None else mesh_seed)
    st, ss, nsf, chi = draw_xs(rng, n_fuel_types, 1, G)
    pin_type = rng.integers(0, n_fuel_types, size=npx * npy)
    xys, tris, mats = [], [], []
    off = 0
    for iy in range(npy):
        for ix in range(npx):
            pxy, ptri, fuel = _pin_template(pitch, r_fuel, m, n_fuel_rings, n_mod_rings, mrng)
            pxy = pxy + np.array([(ix + 0.5) * pitch, (iy + 0.5) * pitch])
            xys.append(pxy)
            tris.append(ptri + off)
            off += len(pxy)
            mats.append(np.where(fuel, pin_type[iy * npx + ix], n_fuel_types))
    xy, tri = _dedup(np.concatenate(xys), np.concatenate(tris))
    W, H = npx * pitch, npy * pitch
    eps = 1e-9
    on_bnd = ((np.abs(xy[:, 0]) < eps) | (np.abs(xy[:, 0] - W) < eps)
              | (np.abs(xy[:, 1]) < eps) | (np.abs(xy[:, 1] - H) < eps))
    if jitter > 0:
        xy = _jitter(xy, tri, ~on_bnd, mrng, jitter)
    mat = np.concatenate(mats).astype(np.int32)
    perm = mrng.permutation(len(tri)).astype(np.int32)   # triangle t -> region perm[t]
    region_material = np.empty(len(tri), np.int32)
    region_material[perm] = mat
    return Problem(name, np.ascontiguousarray(xy), np.ascontiguousarray(tri, np.int32), perm,
                   len(tri), region_material, DOMAIN_BOX, (0.0, 0.0, W, H), 0.0,
                   np.asarray(bc, np.int32), st, ss, nsf, chi, n_azim, n_polar, spacing)


def hex_assembly(*, seed: int, rings: int = 10, pitch: float = 1.6, r_fuel: float = 0.6,
                 gap: float = 0.25, can: float = 0.25, edge: float = 0.0616, G: int = 33,
                 n_fuel_types: int = 3, n_azim: int = 64, n_polar: int = 3,
                 spacing: float = 0.02, jitter: float = 0.10, name: str = "hex") -> Problem:
    """Hexagonal pin lattice (rings rings, 1 + 3 r (r - 1) pins; 10 rings = 271 pins)
    inside a hexagonal can, flats parallel to x, vacuum on the outer hexagon.

    Pin rows are parallel to the flats. The can's inner apothem is the outer pin row's
    distance plus half a pitch plus ``gap``; the wall is ``can`` thick. The domain is
    covered by a regular triangular grid of edge ``edge`` (6 n^2 triangles); grid
    vertices within half an edge of a pin circle (or of the can's inner hexagon) are
    moved onto it, then interior vertices are jittered. Materials by triangle
    centroid: pin fuel (type per pin), coolant, can. Materials are ordered
    [fuel types..., coolant, can].

    Draw order from ``default_rng(seed)``: cross sections (``draw_xs`` with
    Sigma_t ~ U[0.1, 1.5], downscatter band 6, no upscatter), pin fuel types, jitter,
    region numbering."""
    rng = np.random.default_rng(seed)
    st, ss, nsf, chi = draw_xs(rng, n_fuel_types, 2, G, sigt_range=(0.1, 1.5), band=6,
                               upscatter=False)
    nr = rings - 1
    pins = []
    for i in range(-nr, nr + 1):
        for j in range(-nr, nr + 1):
            if max(abs(i), abs(j), abs(i + j)) <= nr:
                pins.append((pitch * (i + 0.5 * j), pitch * (math.sqrt(3) / 2) * j))
    pins = np.array(pins)
    pin_type = rng.integers(0, n_fuel_types, size=len(pins))
    a_in = nr * pitch * math.sqrt(3) / 2 + pitch / 2 + gap
    a_out = a_in + can
    Rc = a_out * 2 / math.sqrt(3)
    n = int(round(Rc / edge))
    s = Rc / n
    e1 = np.array([s, 0.0])
    e2 = np.array([s / 2, s * math.sqrt(3) / 2])
    idx = {}
    pts = []
    for i in range(-n, n + 1):
        for j in range(-n, n + 1):
            if max(abs(i), abs(j), abs(i + j)) <= n:
                idx[(i, j)] = len(pts)
                pts.append(i * e1 + j * e2)
    xy = np.array(pts)
    tris = []
    for i in range(-n - 1, n + 1):
        for j in range(-n - 1, n + 1):
            v, a, b = idx.get((i, j)), idx.get((i + 1, j)), idx.get((i, j + 1))
            c = idx.get((i + 1, j + 1))
            if a is None or b is None:
                continue
            if v is not None:
                tris.append((v, a, b))
            if c is not None:
                tris.append((a, c, b))
    tri = np.array(tris, np.int64)
    # boundary vertices: hex distance == n
    ij = np.array(list(idx.keys()))
    on_bnd = np.max(np.abs(np.stack([ij[:, 0], ij[:, 1], ij[:, 0] + ij[:, 1]], 1)), 1) == n
    # snap to pin circles
    from scipy.spatial import cKDTree
    tree = cKDTree(pins)
    dist, near = tree.query(xy)
    snap = (np.abs(dist - r_fuel) < 0.5 * s) & ~on_bnd
    moved = xy.copy()
    d = xy[snap] - pins[near[snap]]
    moved[snap] = pins[near[snap]] + d / np.linalg.norm(d, axis=1)[:, None] * r_fuel
    # snap to the can's inner hexagon (apothem a_in, normals at 30 + 60k degrees)
    nrm = np.array([[math.cos(math.radians(30 + 60 * k)), math.sin(math.radians(30 + 60 * k))]
                    for k in range(6)])
    proj = xy @ nrm.T
    kmax = np.argmax(proj, axis=1)
    hexd = proj[np.arange(len(xy)), kmax]
    snap2 = (np.abs(hexd - a_in) < 0.5 * s) & ~on_bnd & ~snap
    moved[snap2] = xy[snap2] + (a_in - hexd[snap2])[:, None] * nrm[kmax[snap2]]
    for _ in range(20):
        bad = tri_areas(moved, tri) <= 1e-14
        if not bad.any():
            break
        vb = np.unique(tri[bad].reshape(-1))
        moved[vb] = xy[vb]
    xy = moved
    if jitter > 0:
        xy = _jitter(xy, tri, ~on_bnd, rng, jitter)
    cen = xy[tri].mean(axis=1)
    dist, near = tree.query(cen)
    hexc = np.max(cen @ nrm.T, axis=1)
    mat = np.full(len(tri), n_fuel_types, np.int32)
    fuel = dist < r_fuel
    mat[fuel] = pin_type[near[fuel]]
    mat[hexc > a_in] = n_fuel_types + 1
    perm = rng.permutation(len(tri)).astype(np.int32)
    region_material = np.empty(len(tri), np.int32)
    region_material[perm] = mat
    xy = xy + np.array([Rc, a_out])     # bounding box [0, 2 Rc] x [0, 2 a_out]
    return Problem(name, np.ascontiguousarray(xy), np.ascontiguousarray(tri, np.int32), perm,
                   len(tri), region_material, DOMAIN_HEXAGON, (0.0, 0.0, 2 * Rc, 2 * a_out),
                   a_out, np.full(6, BC_VACUUM, np.int32), st, ss, nsf, chi,
                   n_azim, n_polar, spacing)


def homogenize(p: Problem, material: int = 0) -> Problem:
    """Same mesh, every region assigned one material (infinite-medium tests)."""
    q = dataclasses.replace(p)
    q.region_material = np.full(p.n_regions, material, np.int32)
    return q


def config(cfg: int, seed: Optional[int] = None) -> Problem:
    """The five workload recipes.

    1: single pin cell, 8 regions, 7 groups, A = 16, P = 3, spacing 0.05, reflective.
    2: 17 x 17 square lattice (~31k regions), 7 groups, A = 64, P = 3, 0.02 cm, reflective.
    3: 51 x 51 square lattice (~1.2M regions), 7 groups, A = 128, P = 3, 0.01 cm,
       reflective at x = 0 and y = 0, vacuum at x = W and y = H.
    4: 271-pin hexagonal assembly (~400k regions), 33 groups, A = 64, P = 3, 0.02 cm,
       vacuum.
    5: config-2 geometry (mesh of seed 2) with material map and cross sections drawn
       from ``seed``.
    """
    if cfg == 1:
        return pin_cell_8region(seed=1 if seed is None else seed)
    if cfg == 2:
        return square_lattice(17, 17, seed=2 if seed is None else seed, name="cfg2_17x17")
    if cfg == 3:
        return square_lattice(51, 51, seed=3 if seed is None else seed, m=5, n_fuel_rings=5,
                              n_mod_rings=7, n_azim=128, spacing=0.01,
                              bc=(BC_REFLECTIVE, BC_VACUUM, BC_REFLECTIVE, BC_VACUUM),
                              name="cfg3_51x51")
    if cfg == 4:
        return hex_assembly(seed=4 if seed is None else seed, name="cfg4_hex271")
    if cfg == 5:
        if seed is None:
            raise ValueError("config 5 needs a seed")
        return square_lattice(17, 17, seed=seed, mesh_seed=2, name=f"cfg5_{seed}")
    raise ValueError(f"unknown config {cfg}")


@dataclasses.dataclass
class Extruded:
    """An axially extruded 3D problem (both of the paper's MOC-based 3D methods need
    extruded geometry, Sec. 2.1): the planar problem's mesh, tracking and cross sections
    in every plane, a material per (plane, region), and a boundary condition at the
    bottom and at the top (BC_VACUUM or BC_REFLECTIVE)."""
    name: str
    base: Problem
    dz: np.ndarray              # float64 [Nz] plane heights (cm), bottom to top
    plane_material: np.ndarray  # int32 [Nz, R]
    bc_bottom: int
    bc_top: int

    @property
    def n_planes(self) -> int:
        return int(len(self.dz))


def extrude(p: Problem, dz, plane_material=None, bc_bottom: int = BC_REFLECTIVE,
            bc_top: int = BC_VACUUM, name: Optional[str] = None) -> Extruded:
    """Stack len(dz) planes of the planar problem ``p``. Without ``plane_material`` every
    plane takes the planar material map."""
    dz = np.ascontiguousarray(np.asarray(dz, float).reshape(-1))
    if plane_material is None:
        plane_material = np.tile(p.region_material, (len(dz), 1))
    pm = np.ascontiguousarray(np.asarray(plane_material, np.int32).reshape(len(dz), p.n_regions))
    return Extruded(name or f"{p.name}_x{len(dz)}", p, dz, pm, int(bc_bottom), int(bc_top))


def lattice_with_reflector(p: Problem, n_core: int, n_reflector: int, height: float,
                           bc_bottom: int = BC_REFLECTIVE, bc_top: int = BC_VACUUM,
                           name: Optional[str] = None) -> Extruded:
    """A square lattice extruded into ``n_core`` core planes topped by ``n_reflector``
    planes of moderator (every region takes the moderator, the first non-fuel material),
    all planes of equal height ``height / (n_core + n_reflector)``; the shape of a 3D
    C5G7-type core with an axial water reflector."""
    nz = n_core + n_reflector
    fissile = np.any(p.nu_sigma_f > 0, axis=1)
    moderator = int(np.flatnonzero(~fissile)[0])
    pm = np.tile(p.region_material, (nz, 1))
    pm[n_core:] = moderator
    return extrude(p, np.full(nz, height / nz), pm, bc_bottom, bc_top,
                   name or f"{p.name}_core{n_core}_refl{n_reflector}")


def config_3d(cfg: int) -> Extruded:
    """Extruded workloads for DGMOC.

    6: the config-2 lattice (17 x 17 pins, ~31k regions, 7 groups, A = 64, P = 3,
       0.02 cm) in 12 core planes under 4 moderator-reflector planes, 1.785 cm each
       (28.56 cm), reflective at the bottom and vacuum at the top.
    7: the config-1 pin cell in 4 core planes under 2 reflector planes, 0.5 cm each,
       reflective at the bottom, vacuum at the top (small parity case).
    """
    if cfg == 6:
        return lattice_with_reflector(config(2), 12, 4, 16 * 1.785, name="cfg6_17x17_z16")
    if cfg == 7:
        return lattice_with_reflector(config(1), 4, 2, 3.0, name="cfg7_pin_z6")
    raise ValueError(f"unknown 3D config {cfg}")


def box_problem(W: float = 1.0, H: float = 1.0, nx: int = 2, ny: int = 2, *, G: int = 1,
                sigma_t=None, sigma_s=None, nu_sigma_f=None, chi=None, one_region: bool = False,
                bc=(1, 1, 1, 1), n_azim: int = 16, n_polar: int = 3, spacing: float = 0.05,
                jitter: float = 0.0, seed: int = 0, name: str = "box") -> Problem:
    """Rectangle [0, W] x [0, H] covered by an nx x ny grid of quads, each split into
    two triangles along a seeded random diagonal; one material (index 0) unless the
    caller replaces the map. One triangle per region, or a single region with
    ``one_region``. Default cross sections: a one-group pure absorber, Sigma_t = 1."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0, W, nx + 1)
    ys = np.linspace(0, H, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], 1)
    vid = lambda i, j: j * (nx + 1) + i
    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if rng.random() < 0.5:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    tri = np.array(tris, np.int32)
    on_bnd = ((np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - W) < 1e-12)
              | (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - H) < 1e-12))
    if jitter > 0:
        xy = _jitter(xy, tri, ~on_bnd, rng, jitter)
    if one_region:
        tri_region = np.zeros(len(tri), np.int32)
        R = 1
    else:
        tri_region = np.arange(len(tri), dtype=np.int32)
        R = len(tri)
    st = np.full((1, G), 1.0) if sigma_t is None else np.asarray(sigma_t, float).reshape(-1, G)
    M = st.shape[0]
    ss = np.zeros((M, G, G)) if sigma_s is None else np.asarray(sigma_s, float).reshape(M, G, G)
    nsf = np.zeros((M, G)) if nu_sigma_f is None else np.asarray(nu_sigma_f, float).reshape(M, G)
    ch = np.zeros((M, G)) if chi is None else np.asarray(chi, float).reshape(M, G)
    return Problem(name, np.ascontiguousarray(xy), tri, tri_region, R,
                   np.zeros(R, np.int32), DOMAIN_BOX, (0.0, 0.0, W, H), 0.0,
                   np.asarray(bc, np.int32), st, ss, nsf, ch, n_azim, n_polar, spacing)


def coarse_cells(p: Problem, nx: int, ny: int):
    """Coarse mesh for CMFD: an nx x ny Cartesian grid over the bounding box; each region
    goes to the cell holding its area-weighted centroid, and cells holding no region are
    dropped. For the square lattices with nx, ny = pins per side these are the pin
    cells. Returns (n_cells, region_cell int32 [R])."""
    a = tri_areas(p.xy, p.tri)
    cen = p.xy[p.tri].mean(axis=1)
    R = p.n_regions
    area = np.bincount(p.tri_region, weights=a, minlength=R)
    cx = np.bincount(p.tri_region, weights=a * cen[:, 0], minlength=R) / area
    cy = np.bincount(p.tri_region, weights=a * cen[:, 1], minlength=R) / area
    x0, y0, x1, y1 = p.box
    ix = np.clip(((cx - x0) / (x1 - x0) * nx).astype(np.int64), 0, nx - 1)
    iy = np.clip(((cy - y0) / (y1 - y0) * ny).astype(np.int64), 0, ny - 1)
    raw = iy * nx + ix
    used, region_cell = np.unique(raw, return_inverse=True)
    return int(len(used)), region_cell.astype(np.int32)


def grid_tiles(p: Problem, nx: int, ny: int):
    """Tiles for the tiled DFEM-SN sweep: an nx x ny Cartesian grid over the bounding box;
    each triangle goes to the cell holding its centroid, and cells holding no triangle are
    dropped. On meshes whose edges follow the grid lines (the square lattices with nx, ny =
    pins per side) every tile is a convex cell. Returns (n_tiles, triangle_tile int32 [T])."""
    cen = p.xy[p.tri].mean(axis=1)
    x0, y0, x1, y1 = p.box
    ix = np.clip(((cen[:, 0] - x0) / (x1 - x0) * nx).astype(np.int64), 0, nx - 1)
    iy = np.clip(((cen[:, 1] - y0) / (y1 - y0) * ny).astype(np.int64), 0, ny - 1)
    used, tile = np.unique(iy * nx + ix, return_inverse=True)
    return int(len(used)), tile.astype(np.int32)


# ----------------------------------------------------------------------------------
# coarse brick grids (diffusion HFEM)
# ----------------------------------------------------------------------------------

@dataclasses.dataclass
class BrickGrid:
    """Rectilinear grid of brick nodes with one material per node; node e = (k ny + j) nx + i.
    bc per side x-, x+, y-, y+, z-, z+."""
    name: str
    edges: tuple            # (x_edges, y_edges, z_edges)
    node_material: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    nu_sigma_f: np.ndarray
    chi: np.ndarray
    bc: tuple

    @property
    def n_nodes(self) -> int:
        return int(np.prod([len(e) - 1 for e in self.edges]))

    @property
    def n_groups(self) -> int:
        return int(self.sigma_t.shape[1])


def brick_box(nx: int, ny: int, nz: int, *, G: int, n_fuel: int, n_other: int, seed: int, bc=(1, 1, 1, 1, 1, 1),
              size=(3.0, 2.5, 4.0), jitter: float = 0.3, upscatter: bool = True) -> BrickGrid:
    """Small test grid. Draw order: cross sections (draw_xs), then per axis the node
    widths size / n * U[1 - jitter, 1 + jitter] rescaled to the axis length, then the node
    materials U{0..M-1}."""
    rng = np.random.default_rng(seed)
    st, ss, nsf, chi = draw_xs(rng, n_fuel, n_other, G, upscatter=upscatter)
    edges = []
    for n, L in zip((nx, ny, nz), size):
        w = rng.uniform(1 - jitter, 1 + jitter, n)
        edges.append(np.concatenate([[0.0], np.cumsum(w / w.sum() * L)]))
    mat = rng.integers(0, n_fuel + n_other, nx * ny * nz).astype(np.int32)
    return BrickGrid(f"box{nx}x{ny}x{nz}_g{G}", tuple(edges), mat, st, ss, nsf, chi, tuple(int(b) for b in bc))


def brick_core(n_pins: int = 51, n_fuel_pins: int = 34, pitch: float = 1.26, n_planes: int = 32,
               height: float = 85.68, fuel_height: float = 64.26, G: int = 7, seed: int = 5,
               perturb: float = 0.02) -> BrickGrid:
    """C5G7-like 3D quarter core on pin-cell nodes: n_pins x n_pins pin cells of the given
    pitch, the first n_fuel_pins x n_fuel_pins of them (2 x 2 assemblies of 17 x 17 for the
    defaults) fuel up to fuel_height, the rest moderator; reflective on x-, y-, z- and
    vacuum on x+, y+, z+. Every node carries its own homogenised-like cross sections: the
    base set of its material scaled by 1 + U[-perturb, perturb] (one factor for Sigma_t and
    Sigma_s, one for nuSigma_f), so no two nodes share response matrices.
    Draw order: draw_xs(3 fuel types, moderator, guide tube), fuel type per 17 x 17
    assembly U{0..2}, then the per-node factors; guide tubes sit at the 25 usual
    guide/instrument positions of a 17 x 17 assembly (fixed, not drawn)."""
    rng = np.random.default_rng(seed)
    st0, ss0, nsf0, chi0 = draw_xs(rng, 3, 2, G)
    moderator, guide = 3, 4
    n_asm = max(1, n_fuel_pins // 17)
    asm_type = rng.integers(0, 3, (n_asm, n_asm))
    gt = {(2, 5), (2, 8), (2, 11), (5, 2), (5, 14), (8, 2), (8, 8), (8, 14), (11, 2), (11, 14), (14, 5), (14, 8),
          (14, 11), (3, 3), (3, 13), (13, 3), (13, 13), (5, 5), (5, 11), (11, 5), (11, 11), (5, 8), (8, 5),
          (8, 11), (11, 8)}
    ez = np.linspace(0.0, height, n_planes + 1)
    zc = 0.5 * (ez[:-1] + ez[1:])
    base = np.full((n_planes, n_pins, n_pins), moderator, np.int64)
    for j in range(min(n_fuel_pins, n_pins)):
        for i in range(min(n_fuel_pins, n_pins)):
            m = guide if (i % 17, j % 17) in gt else int(asm_type[min(j // 17, n_asm - 1), min(i // 17, n_asm - 1)])
            base[zc < fuel_height, j, i] = m
    base = base.ravel()
    N = base.size
    f_t = 1.0 + rng.uniform(-perturb, perturb, N)
    f_f = 1.0 + rng.uniform(-perturb, perturb, N)
    st = st0[base] * f_t[:, None]
    ss = ss0[base] * f_t[:, None, None]
    nsf = nsf0[base] * f_f[:, None]
    chi = chi0[base].copy()
    edges = (np.arange(n_pins + 1) * pitch, np.arange(n_pins + 1) * pitch, ez)
    return BrickGrid(f"core{n_pins}x{n_pins}x{n_planes}_g{G}", edges, np.arange(N, dtype=np.int32), st, ss, nsf, chi,
                     (BC_REFLECTIVE, BC_VACUUM, BC_REFLECTIVE, BC_VACUUM, BC_REFLECTIVE, BC_VACUUM))
