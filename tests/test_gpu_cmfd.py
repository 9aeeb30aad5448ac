"""CMFD on the GPU against the CMFD oracle, through the C ABI.

* Surface currents of one sweep: net current per coarse surface against the oracle's
  partial-current tallies (FP64 to 1e-10, FP32 to 2e-5 of the largest current), and the
  scalar flux of the current-tallying sweep variant against the oracle as for the plain
  sweep.
* One CMFD-accelerated power iteration from the cold start, with the coarse eigenproblem
  converged tightly on the device, against the oracle's (direct sparse solves) to 1e-8.
* Accelerated solves reach the plain power iteration's fixed point in fewer sweeps.
"""
import sys

import numpy as np
import pytest

from oracle import cmfd_oracle as CM
from oracle.oracle import Oracle
from paper_2607_01591_amd import moc
from paper_2607_01591_amd import problems as P

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(x, ref):
    m = ref > 1e-12 * ref.max()
    return float(np.max(np.abs(x[m] - ref[m]) / ref[m]))


def _dev(a, cuda):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=cuda)


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_surface_currents(o):
    """Net currents per surface (a, b), a < b or b = -1, from the oracle's partials."""
    off, nbr = o.coarse_adjacency()
    jp, jin = o.currents()
    J = CM.net_currents(off, nbr, jp, jin)
    out = {}
    for i in range(len(off) - 1):
        for s in range(off[i], off[i + 1]):
            j = int(nbr[s])
            if j < 0:
                out[(i, -1)] = J[s]
            elif i < j:
                out[(i, j)] = J[s]
    return out


CASES = [
    ("lattice3x3_vacuum2", lambda: P.square_lattice(3, 3, seed=1, n_azim=16, spacing=0.05, bc=(1, 0, 1, 0)), (3, 3)),
    ("lattice4x4_cells2x2", lambda: P.square_lattice(4, 4, seed=6, n_azim=8, spacing=0.08, bc=(0, 0, 0, 0)), (2, 2)),
    ("hex_small_grid4", lambda: P.hex_assembly(seed=5, rings=3, edge=0.25, G=4, spacing=0.05, n_azim=16), (4, 4)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,make,grid", CASES, ids=[c[0] for c in CASES])
def test_surface_currents_match_oracle(name, make, grid, precision, cuda):
    log(f"[cmfd currents] {name} {precision}")
    prob = make()
    n, rc = P.coarse_cells(prob, *grid)
    o = Oracle.from_problem(prob)
    o.set_coarse(n, rc)
    s = moc.Solver(prob, precision=precision)
    s.set_coarse_mesh(n, rc)
    rng = np.random.default_rng(5)
    src = rng.uniform(0.1, 2.0, size=(o.R, o.G))
    psi0 = rng.uniform(0.0, 1.0, size=o.psi_shape())
    if precision == "f32":
        psi0 = psi0.astype(np.float32).astype(np.float64)
    o.set_psi(psi0)
    phi_ref = o.sweep(src)
    ref = oracle_surface_currents(o)
    s.set_boundary_flux(_dev(psi0, cuda))
    phi = _host(s.sweep(_dev(src, cuda)))
    cells, cur = s.surface_currents()
    got = {(int(a), int(b)): cur[i] for i, (a, b) in enumerate(cells)}
    assert set(got) == set(ref)
    scale = max(np.abs(v).max() for v in ref.values())
    tol = 1e-10 if precision == "f64" else 2e-5
    worst = max(np.abs(got[k] - ref[k]).max() for k in ref) / scale
    log(f"  {len(ref)} surfaces, worst |dJ| / max|J| = {worst:.2e}")
    assert worst < tol
    assert rel_err(phi, phi_ref) < (1e-11 if precision == "f64" else 1e-5)


@pytest.mark.parametrize("blocks", [1, 3], ids=["one_workgroup", "grid3"])
@pytest.mark.parametrize("name,make,grid", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_one_cmfd_iteration_matches_oracle(name, make, grid, blocks, cuda):
    """Both coarse-solve paths (one workgroup; a cooperative grid of blocks)."""
    log(f"[cmfd one iteration] {name} blocks={blocks}")
    prob = make()
    n, rc = P.coarse_cells(prob, *grid)
    ref = CM.solve(Oracle.from_problem(prob), prob, tol=1e-30, max_iter=2, n_cells=n, region_cell=rc,
                   history=True)
    s = moc.Solver(prob, precision="f64")
    s.set_coarse_mesh(n, rc, tol=1e-11, max_outer=500, max_inner=500, coarse_blocks=blocks)
    for it in (1, 2):
        r = s.run_iterations(it)
        phi = _host(s.flux())
        h = ref["history"][it - 1]
        info = s.coarse_info()
        log(f"  iteration {it}: k {r['k']:.12f} vs {h['k']:.12f}; coarse {info['last_outer']} outer, "
            f"{info['last_inner']} inner")
        assert abs(r["k"] - h["k"]) < 1e-9
        assert rel_err(phi, h["phi"]) < 1e-8


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cmfd_reaches_plain_fixed_point_in_fewer_sweeps(precision, cuda):
    log(f"[cmfd fixed point] {precision}")
    prob = P.square_lattice(6, 6, seed=9, n_azim=16, spacing=0.05, bc=(1, 0, 1, 0))
    n, rc = P.coarse_cells(prob, 6, 6)
    s = moc.Solver(prob, precision=precision, max_iter=5000)
    tol = 1e-9 if precision == "f64" else 1e-6
    plain = s.solve(tol)
    phi_plain = _host(s.flux())
    s.set_coarse_mesh(n, rc)
    acc = s.solve(tol)
    phi_acc = _host(s.flux())
    log(f"  plain {plain['iterations']} iterations, CMFD {acc['iterations']} (k {plain['k']:.9f} / {acc['k']:.9f})")
    assert plain["converged"] and acc["converged"]
    assert acc["iterations"] * 3 < plain["iterations"]
    if precision == "f64":
        assert abs(acc["k"] - plain["k"]) < 1e-8
        assert rel_err(phi_acc, phi_plain) < 1e-6
    else:
        # both stop at a 1e-6 residual of a slowly converging FP32 iteration
        assert abs(acc["k"] - plain["k"]) < 2e-5
        assert rel_err(phi_acc, phi_plain) < 2e-3
    # removing the coarse mesh restores the plain iteration (tally atomics make the last
    # bits order-dependent, so allow an iteration of slack)
    s.set_coarse_mesh(0)
    again = s.solve(tol)
    assert abs(again["iterations"] - plain["iterations"]) <= 1
    assert abs(again["k"] - plain["k"]) < (1e-11 if precision == "f64" else 1e-6)


@pytest.mark.parametrize("blocks", [0, 2])
def test_cmfd_solution_matches_oracle_fixed_point(blocks, cuda):
    """FP64 CMFD solve against the oracle's plain power iteration at a tight tolerance."""
    log(f"[cmfd vs oracle fixed point] blocks={blocks}")
    prob = P.square_lattice(3, 3, seed=2, n_azim=16, spacing=0.05, bc=(1, 0, 1, 0))
    n, rc = P.coarse_cells(prob, 3, 3)
    ref = Oracle.from_problem(prob).solve(tol=1e-10, max_iter=5000)
    s = moc.Solver(prob, precision="f64")
    s.set_coarse_mesh(n, rc, coarse_blocks=blocks)
    r = s.solve(1e-10)
    assert r["converged"]
    assert abs(r["k"] - ref["k"]) < 1e-8
    assert rel_err(_host(s.flux()), ref["phi"]) < 1e-7


def test_cmfd_grid_and_workgroup_paths_agree_on_a_larger_lattice(cuda):
    """17 x 17 pin cells (2023 coarse unknowns): the cooperative-grid coarse solve and the
    one-workgroup solve reach the same converged answer."""
    log("[cmfd grid vs workgroup] 17x17")
    prob = P.config(2)
    n, rc = P.coarse_cells(prob, 17, 17)
    s = moc.Solver(prob, precision="f64", max_iter=5000)
    out = {}
    for blocks in (1, 8):
        s.set_coarse_mesh(n, rc, coarse_blocks=blocks)
        r = s.solve(1e-9)
        assert r["converged"]
        out[blocks] = (r, _host(s.flux()))
        log(f"  blocks {blocks}: {r['iterations']} iterations, k {r['k']:.10f}, {r['wall_ms']:.0f} ms")
    assert abs(out[1][0]["k"] - out[8][0]["k"]) < 1e-9
    assert rel_err(out[8][1], out[1][1]) < 1e-7
