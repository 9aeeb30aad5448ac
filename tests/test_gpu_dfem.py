"""DFEM-SN on the GPU against the FP64 DFEM-SN oracle, through the C ABI.

* Four consecutive sweeps from the cold state with random emission moments (slopes
  included; each takes its reflective inflow from the one before; the last two replay
  the recorded sweep graphs), over problems
  with vacuum, reflective and mixed sides, 1 to 4 polar angles and 1 to 7 groups. FP64
  to 1e-11, FP32 to 1e-5, relative to the largest element average of the group.
* Converged eigenvalue and fixed-source solves against the oracle's.
* The 17 x 17 lattice mesh in the timed launch configuration (64 azimuths x 3 polar,
  7 groups, FP32), homogenised, purely absorbing, reflective, with a flat source: the
  exact solution is q / Sigma_t in every element with zero slopes.
* Tiled sweeps (moc_sn_set_tiles) against level-by-level sweeps, bit for bit, for three
  sweeps in a row, FP64 and FP32: one tile for the whole domain, one tile per element
  (every flux passes through storage slots), grid tiles on an unjittered box and on the
  pin cell's quadrants, and the 17 x 17 pin-cell tiles of the lattice mesh; a tiled
  eigenvalue solve against the oracle's.
"""
import sys

import numpy as np
import pytest

from oracle import sn_oracle as SN
from paper_2607_01591_amd import dfem
from paper_2607_01591_amd import problems as P

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, cuda):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=cuda)


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def moment_err(x, ref):
    scale = np.abs(ref[..., 0]).max(axis=0)      # [G]
    return float((np.abs(x - ref) / scale[None, :, None]).max())


def box(G, Pn, bc, seed, n=6, A=8, jitter=0.1):
    rng = np.random.default_rng(seed)
    st, ss, nsf, chi = P.draw_xs(rng, 1, 2, G)
    p = P.box_problem(1.2, 0.9, n, n - 1, G=G, sigma_t=st, sigma_s=ss, nu_sigma_f=nsf, chi=chi, bc=bc,
                      n_azim=A, n_polar=Pn, spacing=0.1, jitter=jitter, seed=seed)
    p.region_material = rng.integers(0, 3, p.n_regions).astype(np.int32)
    return p


CASES = [
    ("pincell_reflective", lambda: P.pin_cell_8region(seed=1, n_azim=8, n_polar=2)),
    ("box_g2_p2_mixed", lambda: box(2, 2, (1, 0, 1, 0), 1)),
    ("box_g3_p3_vacuum", lambda: box(3, 3, (0, 0, 0, 0), 2)),
    ("box_g4_p4_reflective", lambda: box(4, 4, (1, 1, 1, 1), 3, A=12)),
    ("box_g1_p1_mixed", lambda: box(1, 1, (0, 1, 1, 0), 4, A=16)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sweeps_match_oracle(name, make, precision, cuda):
    log(f"[dfem sweeps] {name} {precision}")
    prob = make()
    o = SN.SNOracle(prob)
    s = dfem.SNSolver(prob, precision=precision)
    rng = np.random.default_rng(8)
    tol = 1e-11 if precision == "f64" else 1e-5
    for k in range(4):   # sweeps 3 and 4 replay the recorded sweep graphs
        src = rng.uniform(0.1, 2.0, o.shape())
        src[..., 1:] = rng.uniform(-0.5, 0.5, src[..., 1:].shape)
        ref = o.sweep(src)
        got = _host(s.sweep(_dev(src, cuda)))
        err = moment_err(got, ref)
        log(f"  sweep {k + 1}: error {err:.2e} ({s.info})")
        assert err < tol


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eigen_solve_matches_oracle(precision, cuda):
    log(f"[dfem eigen] {precision}")
    prob = P.pin_cell_8region(seed=1, n_azim=16, n_polar=3)
    ref = SN.SNOracle(prob).solve(tol=1e-10, max_iter=5000)
    s = dfem.SNSolver(prob, precision=precision, max_iter=5000)
    r = s.solve(1e-10 if precision == "f64" else 1e-6)
    err = moment_err(_host(s.flux()), ref["phi"])
    log(f"  k {r['k']:.12f} vs {ref['k']:.12f}; {r['iterations']} vs {ref['iterations']} iterations; error {err:.2e}")
    assert r["converged"] and ref["converged"]
    if precision == "f64":
        assert abs(r["k"] - ref["k"]) < 1e-9 and err < 1e-7
    else:
        assert abs(r["k"] - ref["k"]) < 1e-5 and err < 1e-4


def test_fixed_source_solve_matches_oracle(cuda):
    log("[dfem fixed source] f32")
    prob = box(2, 2, (1, 0, 1, 0), 6)
    prob.nu_sigma_f[:] = 0.0
    o = SN.SNOracle(prob)
    rng = np.random.default_rng(3)
    q = np.zeros(o.shape())
    q[..., 0] = rng.uniform(0.0, 1.0, q[..., 0].shape)
    q[..., 1:] = rng.uniform(-0.2, 0.2, q[..., 1:].shape)
    o.set_external_source(q)
    ref = o.solve(tol=1e-11, max_iter=5000)
    s = dfem.SNSolver(prob, precision="f32", max_iter=5000)
    s.set_external_source(_dev(q, cuda))
    r = s.solve(1e-7)
    err = moment_err(_host(s.flux()), ref["phi"])
    log(f"  {r['iterations']} iterations, error {err:.2e}")
    assert r["converged"] and ref["converged"] and err < 2e-5


def test_full_size_absorber_is_flat(cuda):
    """17 x 17 lattice mesh (31,212 triangles), 64 x 3 directions, 7 groups, FP32."""
    import dataclasses
    base = P.homogenize(P.config(2), 0)
    prob = dataclasses.replace(base, sigma_s=np.zeros_like(base.sigma_s), nu_sigma_f=np.zeros_like(base.nu_sigma_f),
                               chi=np.zeros_like(base.chi))
    s = dfem.SNSolver(prob, precision="f32", max_iter=200)
    log(f"[dfem full size absorber] {s.info}")
    G = prob.n_groups
    q = np.zeros(s.shape())
    q[..., 0] = np.linspace(0.5, 1.5, G)[None, :]
    s.set_external_source(_dev(q, cuda))
    r = s.solve(1e-7)
    phi = _host(s.flux())
    exact = q[0, :, 0] / prob.sigma_t[0]
    err0 = float(np.abs(phi[..., 0] / exact[None, :] - 1).max())
    err1 = float(np.abs(phi[..., 1:]).max() / exact.max())
    log(f"  {r['iterations']} iterations ({r['wall_ms']:.0f} ms): average error {err0:.2e}, slopes {err1:.2e}")
    assert r["converged"] and err0 < 1e-5 and err1 < 1e-5


def _tiled_pair(prob, precision, tile, cuda, n=3, seed=11):
    """Level-by-level and tiled sweeps of the same emission, n in a row (reflective inflow
    from the sweep before): the fluxes must agree bit for bit."""
    a = dfem.SNSolver(prob, precision=precision)
    b = dfem.SNSolver(prob, precision=precision)
    b.set_tiles(tile)
    assert b.info["n_tiles"] == int(tile.max()) + 1 and a.info["n_tiles"] == 0
    rng = np.random.default_rng(seed)
    for k in range(n):
        src = rng.uniform(0.1, 2.0, a.shape())
        src[..., 1:] = rng.uniform(-0.5, 0.5, src[..., 1:].shape)
        sd = _dev(src, cuda)
        ga, gb = _host(a.sweep(sd)), _host(b.sweep(sd))
        diff = int((ga != gb).sum())
        log(f"  sweep {k + 1}: {diff} of {ga.size} entries differ ({b.info['n_tiles']} tiles, "
            f"{b.info['n_tile_levels']} tile levels, {b.info['n_tile_slots']} slots)")
        assert np.isfinite(gb).all() and diff == 0
    return b


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_tiled_sweeps_equal_levels(name, make, precision, cuda):
    log(f"[dfem tiles] {name} {precision}")
    prob = make()
    T = len(prob.tri)
    tilings = [("per element", np.arange(T, dtype=np.int32))]
    if name == "pincell_reflective":
        tilings.append(("quadrants", P.grid_tiles(prob, 2, 2)[1]))
    else:
        tilings.append(("whole domain", np.zeros(T, np.int32)))
    for what, tile in tilings:
        log(f" {what}")
        _tiled_pair(prob, precision, tile, cuda)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tiled_grid_on_unjittered_box(precision, cuda):
    prob = box(3, 2, (1, 0, 1, 1), 5, n=6, A=12, jitter=0.0)
    for nx, ny in ((3, 5), (2, 1), (6, 5)):
        log(f"[dfem tiles] unjittered box, {nx} x {ny} grid tiles, {precision}")
        _tiled_pair(prob, precision, P.grid_tiles(prob, nx, ny)[1], cuda)


def test_tiled_full_size(cuda):
    """17 x 17 lattice mesh, 64 x 3 directions, 7 groups, pin-cell tiles: FP32 and FP64."""
    prob = P.config(2)
    n, tile = P.grid_tiles(prob, 17, 17)
    assert n == 289
    log("[dfem tiles] 17x17 lattice, pin-cell tiles, f32")
    b = _tiled_pair(prob, "f32", tile, cuda, n=2)
    assert b.info["n_tile_levels"] == 33 and b.info["n_levels"] == 797
    log("[dfem tiles] 17x17 lattice, pin-cell tiles, f64")
    _tiled_pair(prob, "f64", tile, cuda, n=1)


def test_tiled_eigen_solve_matches_oracle(cuda):
    log("[dfem tiles] eigen solve, pin cell quadrants, f64")
    prob = P.pin_cell_8region(seed=1, n_azim=16, n_polar=3)
    ref = SN.SNOracle(prob).solve(tol=1e-10, max_iter=5000)
    s = dfem.SNSolver(prob, precision="f64", max_iter=5000)
    s.set_tiles(P.grid_tiles(prob, 2, 2)[1])
    r = s.solve(1e-10)
    err = moment_err(_host(s.flux()), ref["phi"])
    log(f"  k {r['k']:.12f} vs {ref['k']:.12f}; error {err:.2e}")
    assert r["converged"] and abs(r["k"] - ref["k"]) < 1e-9 and err < 1e-7
