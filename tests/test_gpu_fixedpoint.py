"""Converged parity at the benchmarked sizes: a fixed-point check against the FP64 oracle.

A cold FP32 solve of the workload runs on the GPU past its own stopping point; its
converged state (scalar flux phi, eigenvalue k and the incoming boundary angular fluxes)
is handed to the oracle, which runs three FP64 power iterations from it (the iteration
that defines k_eff of Eq. MGNTE, Sec. 2, with every sweep by Eq. MOC_sol, Sec. 2.1). At a
fixed point of the discrete FP64 equations those iterations barely move. Required, as
stated per result:

* oracle residual of its last iteration (volume-weighted L2 step of phi) < 1e-6;
* largest relative change of phi over the three iterations < 1e-5 (over (r, g) with
  phi above 1e-12 of its maximum);
* |k_oracle - k_gpu| < 1e-5.

Workloads: the 17 x 17 lattice (three seeds), the 271-pin hexagon with 33 groups (group
batches of 8 in the sweep), the 51 x 51 lattice (solved with CMFD on its pin cells; the
converged answer is the plain iteration's), and one warm-started solve of the
warm-start family (network guess, then the plain iteration).
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2607_01591_amd import moc
from paper_2607_01591_amd import problems as P

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
RES_TOL, MOVE_TOL, DK_TOL = 1e-6, 1e-5, 1e-5
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2607_01591_amd", "weights", "warmstart_17x17.npz")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def converge(s, tol=1e-6, extra=0.5):
    """Solve to tol, then repeat the same cold-started iteration for (1 + extra) times as
    many iterations, which takes the FP32 iterate past the stopping point towards its
    own rounding floor. Returns the result of the longer run."""
    r = s.solve(tol)
    assert r["converged"], r
    n = int(r["iterations"] * (1.0 + extra)) + 1
    return s.run_iterations(n)


def fixed_point_check(prob, s, k, label, iters=3):
    phi = s.flux().cpu().numpy()
    psi = s.get_boundary_flux().cpu().numpy()
    t0 = time.perf_counter()
    o = Oracle.from_problem(prob, threads=THREADS)
    o.set_threads(THREADS)
    t1 = time.perf_counter()
    o.set_psi(psi)
    V = o.volumes()
    nsf = prob.nu_sigma_f[prob.region_material]
    start = phi / np.sum(V[:, None] * nsf * phi)      # the oracle's own normalisation
    r = o.solve(tol=0.0, max_iter=iters, phi0=phi, k0=k)
    t2 = time.perf_counter()
    ref = r["phi"]
    m = ref > 1e-12 * ref.max()
    move = float(np.max(np.abs(start[m] - ref[m]) / ref[m]))
    dk = abs(r["k"] - k)
    log(f"  {label}: oracle after {iters} iterations: residual {r['residual']:.2e}, "
        f"max rel phi move {move:.2e}, |dk| {dk:.2e} (k gpu {k:.8f}, oracle {r['k']:.8f}); "
        f"oracle setup {t1 - t0:.1f} s, iterations {t2 - t1:.1f} s on {THREADS} threads")
    assert r["residual"] < RES_TOL
    assert move < MOVE_TOL
    assert dk < DK_TOL
    return r, move


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_lattice17_fixed_point(seed, cuda):
    log(f"[fixed point] 17x17 lattice, seed {seed}")
    prob = P.config(2, seed=seed)
    s = moc.Solver(prob, precision="f32", max_iter=20000, check_every=10)
    r = converge(s)
    log(f"  GPU FP32: {r['iterations']} iterations, residual {r['residual']:.2e}, k {r['k']:.8f}")
    fixed_point_check(prob, s, r["k"], "17x17")


def test_hexagon_g33_fixed_point(cuda):
    import torch
    log("[fixed point] 271-pin hexagon, 33 groups")
    prob = P.config(4)
    s = moc.Solver(prob, precision="f32", max_iter=20000, check_every=10)
    r = converge(s)
    log(f"  GPU FP32: {r['iterations']} iterations, residual {r['residual']:.2e}, k {r['k']:.8f}")
    fixed_point_check(prob, s, r["k"], "hexagon")
    del s
    torch.cuda.empty_cache()


def test_lattice51_fixed_point(cuda):
    import torch
    log("[fixed point] 51x51 lattice (CMFD-accelerated GPU solve)")
    prob = P.config(3)
    s = moc.Solver(prob, precision="f32", max_iter=2000, check_every=1)
    n_cells, region_cell = P.coarse_cells(prob, 51, 51)
    s.set_coarse_mesh(n_cells, region_cell)
    r = s.solve(1e-7)
    log(f"  GPU FP32 + CMFD: {r['iterations']} iterations, residual {r['residual']:.2e}, k {r['k']:.8f}")
    assert r["converged"]
    fixed_point_check(prob, s, r["k"], "51x51")
    del s
    torch.cuda.empty_cache()


def test_warm_started_fixed_point(cuda):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained warm-start weights in the tree")
    from paper_2607_01591_amd.warmstart import WarmStart, load_net
    log("[fixed point] warm-started 17x17 problem (held-out seed 200003)")
    base = P.config(5, seed=100000)
    s = moc.Solver(base, precision="f32", max_iter=20000, check_every=10)
    ws = WarmStart(s, base, cuda, net=load_net(WEIGHTS, cuda, base.n_groups))
    p = P.config(5, seed=200003)
    s.set_materials(p)
    w = ws.solve_warm(p, 1e-6)
    log(f"  GPU FP32 warm: {w['sweeps']} sweeps, residual {w['residual']:.2e}, k {w['k']:.8f}")
    assert w["converged"] and not w["flags"] & moc.FLAG_FELL_BACK_TO_COLD
    # continue the same iteration past its stopping point, as for the cold solves: the
    # converged state is handed back as a guess (flux, k and boundary fluxes)
    s.set_initial_guess(s.flux(), w["k"], s.get_boundary_flux())
    r = s.run_iterations(w["iterations"] // 2 + 1)
    log(f"  continued {r['iterations']} iterations: residual {r['residual']:.2e}, k {r['k']:.8f}")
    assert not r["flags"] & moc.FLAG_FELL_BACK_TO_COLD
    fixed_point_check(p, s, r["k"], "warm 17x17")
