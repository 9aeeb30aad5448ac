"""DGMOC on the GPU against the FP64 DGMOC oracle, through the C ABI.

* Sweeps: two consecutive sweeps from the cold state with random emission moments (the
  second one carries the radial boundary fluxes and the bottom-face buffer of the
  first), over problems with every combination of axial boundary conditions, 1 to 4
  polar angles, 1, 2 and 4 groups per wavefront (ragged group batches), and angle blocks
  of one angle, a few angles and all angles. FP64 instantiation to 1e-11, FP32 to 1e-5,
  both relative to the largest plane-average flux of the group.
* Converged eigenvalue and fixed-source solves against the oracle's.
* The extruded 17 x 17 workload (the launch configuration that is timed), homogenised
  and reflective everywhere: the exact fixed point is flat with k = k-infinity.
"""
import sys

import numpy as np
import pytest

from oracle.dg_oracle import DGOracle
from paper_2607_01591_amd import dgmoc
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
    """max |x - ref| over both moments, relative to the largest |plane average| of the
    same group (the P1 moment changes sign, so elementwise relative errors are
    meaningless for it)."""
    scale = np.abs(ref[..., 0]).max(axis=(0, 1))          # [G]
    return float((np.abs(x - ref) / scale[None, None, :, None]).max())


def box3(G, n_polar, bc_bot, bc_top, seed=0):
    """A 3 x 2 box with three materials in a pattern that changes with height."""
    rng = np.random.default_rng(seed)
    st, ss, nsf, chi = P.draw_xs(rng, 1, 2, G)
    base = P.box_problem(1.1, 0.8, 3, 2, G=G, sigma_t=st, sigma_s=ss, nu_sigma_f=nsf, chi=chi, bc=(1, 0, 1, 1),
                         n_azim=8, n_polar=n_polar, spacing=0.06, jitter=0.1, seed=seed)
    R = base.n_regions
    pm = np.stack([rng.integers(0, 3, R) for _ in range(3)]).astype(np.int32)
    pm[:, 0] = 0
    return P.extrude(base, [0.35, 0.6, 0.45], pm, bc_bottom=bc_bot, bc_top=bc_top)


CASES = [
    ("pin_reflector_z6", lambda: P.config_3d(7), dict()),
    ("pin_reflector_z6_block1", lambda: P.config_3d(7), dict(angle_block=1)),
    ("box_g3_p2_vac_vac_gb2", lambda: box3(3, 2, P.BC_VACUUM, P.BC_VACUUM), dict(group_batch=2)),
    ("box_g5_p4_refl_refl_block3", lambda: box3(5, 4, P.BC_REFLECTIVE, P.BC_REFLECTIVE), dict(angle_block=3)),
    ("box_g2_p1_vac_refl_gb1", lambda: box3(2, 1, P.BC_VACUUM, P.BC_REFLECTIVE), dict(group_batch=1)),
    ("box_g7_p3_refl_vac_gb4_slots64", lambda: box3(7, 3, P.BC_REFLECTIVE, P.BC_VACUUM, seed=3),
     dict(group_batch=4, tally_slots=64)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_two_sweeps_match_oracle(name, make, opts, precision, cuda):
    log(f"[dgmoc sweeps] {name} {precision}")
    ext = make()
    o = DGOracle(ext)
    s = dgmoc.DGSolver(ext, precision=precision, **opts)
    rng = np.random.default_rng(7)
    tol = 1e-11 if precision == "f64" else 1e-5
    for k in range(2):
        src = rng.uniform(0.1, 2.0, o.flux_shape())
        src[..., 1] = rng.uniform(-0.5, 0.5, src[..., 1].shape)
        ref = o.sweep(src)
        got = _host(s.sweep(_dev(src, cuda)))
        err = moment_err(got, ref)
        log(f"  sweep {k + 1}: max error {err:.2e} (info {s.info})")
        assert err < tol


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eigen_solve_matches_oracle(precision, cuda):
    log(f"[dgmoc eigen] {precision}")
    ext = P.config_3d(7)
    ref = DGOracle(ext).solve(tol=1e-10, max_iter=20000)
    s = dgmoc.DGSolver(ext, precision=precision, max_iter=20000)
    tol = 1e-10 if precision == "f64" else 1e-6
    r = s.solve(tol)
    phi = _host(s.flux())
    err = moment_err(phi, ref["phi"])
    log(f"  k {r['k']:.12f} vs {ref['k']:.12f}; {r['iterations']} vs {ref['iterations']} iterations; flux error {err:.2e}")
    assert r["converged"] and ref["converged"]
    if precision == "f64":
        assert abs(r["k"] - ref["k"]) < 1e-9
        assert err < 1e-7
    else:
        assert abs(r["k"] - ref["k"]) < 1e-5
        assert err < 1e-4


def test_fixed_source_solve_matches_oracle(cuda):
    log("[dgmoc fixed source] f32")
    ext = box3(2, 2, P.BC_REFLECTIVE, P.BC_VACUUM, seed=5)
    ext.base.nu_sigma_f[:] = 0.0
    o = DGOracle(ext)
    rng = np.random.default_rng(2)
    q = np.zeros(o.flux_shape())
    q[..., 0] = rng.uniform(0.0, 1.0, q[..., 0].shape)
    q[..., 1] = rng.uniform(-0.2, 0.2, q[..., 1].shape)
    o.set_external_source(q)
    ref = o.solve(tol=1e-11, max_iter=20000)
    s = dgmoc.DGSolver(ext, precision="f32", max_iter=20000)
    s.set_external_source(_dev(q, cuda))
    r = s.solve(1e-7)
    err = moment_err(_host(s.flux()), ref["phi"])
    log(f"  {r['iterations']} iterations, flux error {err:.2e}")
    assert r["converged"] and ref["converged"]
    assert err < 2e-5


def test_angle_blocks_do_not_change_the_answer(cuda):
    """Sequential angle blocks (Alg. DGMOC_sweep) and one block holding every angle give
    the same sweep up to summation order."""
    ext = P.config_3d(7)
    rng = np.random.default_rng(4)
    src = rng.uniform(0.1, 1.0, (ext.n_planes, ext.base.n_regions, ext.base.n_groups, 2))
    out = {}
    for blk in (0, 1, 3):
        s = dgmoc.DGSolver(ext, precision="f64", angle_block=blk)
        out[blk] = [_host(s.sweep(_dev(src, cuda))) for _ in range(2)]
    for blk in (1, 3):
        for k in range(2):
            assert moment_err(out[blk][k], out[0][k]) < 1e-12


def radially_uniform(ext, scatter_scale=0.35):
    """The same planes, radially uniform: every region of plane z takes one material
    (core planes 0, 1 in the lower and upper halves of the core, reflector 2), with the
    scattering scaled down (ratio <= 0.33) and no fission: a fixed-source problem whose
    source iteration converges in a few tens of sweeps."""
    import dataclasses
    base = ext.base
    nz = ext.n_planes
    n_core = int(np.sum(np.any(base.nu_sigma_f[ext.plane_material] > 0, axis=(1, 2))))
    mats = np.array([0 if z < n_core // 2 else 1 if z < n_core else 2 for z in range(nz)], np.int32)
    b2 = dataclasses.replace(base, sigma_s=base.sigma_s * scatter_scale, nu_sigma_f=np.zeros_like(base.nu_sigma_f),
                             chi=np.zeros_like(base.chi))
    pm = np.repeat(mats[:, None], base.n_regions, axis=1)
    return P.extrude(b2, ext.dz, pm, bc_bottom=ext.bc_bottom, bc_top=ext.bc_top), mats


def test_full_size_radially_uniform_slab(cuda):
    """The extruded 17 x 17 workload (16 planes, bottom reflective, top vacuum) in the
    timed launch configuration (FP32, default options), made radially uniform per plane
    with reflective sides and a plane-wise source (both moments): the exact discrete
    solution is flat in every plane and equals the 1D slab solution, taken here from the
    DGMOC oracle on a one-cell box with the same planes and polar quadrature."""
    ext, mats = radially_uniform(P.config_3d(6))
    G, nz = ext.base.n_groups, ext.n_planes
    rng = np.random.default_rng(11)
    qz = np.zeros((nz, G, 2))
    qz[:12, :, 0] = rng.uniform(0.5, 1.5, (12, G))
    qz[:12, :, 1] = rng.uniform(-0.3, 0.3, (12, G))
    tiny = P.box_problem(1.0, 1.0, 1, 1, G=G, sigma_t=ext.base.sigma_t, sigma_s=ext.base.sigma_s,
                         nu_sigma_f=ext.base.nu_sigma_f, chi=ext.base.chi, bc=(1, 1, 1, 1), n_azim=8,
                         n_polar=ext.base.n_polar, spacing=0.3, one_region=True)
    tiny_ext = P.extrude(tiny, ext.dz, mats[:, None], bc_bottom=ext.bc_bottom, bc_top=ext.bc_top)
    o = DGOracle(tiny_ext)
    o.set_external_source(qz[:, None, :, :])
    ref = o.solve(tol=1e-12, max_iter=5000)
    assert ref["converged"]
    ref_z = ref["phi"][:, 0]                                   # [Nz, G, 2]
    log(f"[dgmoc full size slab] oracle: {ref['iterations']} iterations")
    s = dgmoc.DGSolver(ext, precision="f32", max_iter=500)
    q = np.broadcast_to(qz[:, None, :, :], s.shape()).copy()
    s.set_external_source(_dev(q, cuda))
    r = s.solve(1e-7)
    phi = _host(s.flux())
    err = moment_err(phi, np.broadcast_to(ref_z[:, None], phi.shape))
    log(f"  GPU {r['iterations']} iterations ({r['wall_ms']:.0f} ms, {s.info}); error {err:.2e}")
    assert r["converged"]
    assert err < 2e-5
