"""Parity at the benchmarked sizes, in the launch configuration bench.py times.

* 17 x 17 lattice (31k regions, 12.3M segments) and the 271-pin hexagon (399k regions,
  33 groups, the group-batch-11 sweep instance): one FP32 sweep against one oracle sweep,
  element by element.
* 51 x 51 lattice (1.2M regions, 1.0e9 segments) and the hexagon again: the per-group
  balance identity of a sweep
      sum_r V_r (Sigma_t phi_r - s_r) = sum_{tracks, senses, polar} c_ap (psi_in - psi_out)
  (every increment is tallied exactly once, with the right weight), and agreement of
  the FP32 sweep with its FP64 instantiation. The converged answers of these workloads are
  checked against the oracle by the fixed-point tests.
"""
import math
import sys

import numpy as np
import pytest

from paper_2607_01591_amd import moc
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


def _sweep(s, src_d, psi_d, cuda):
    import torch
    s.set_boundary_flux(psi_d)
    ex = torch.zeros(s.psi_shape(), dtype=torch.float64, device=cuda)
    s.set_exit_buffer(ex)
    phi = s.sweep(src_d)
    torch.cuda.synchronize()
    s.set_exit_buffer(None)
    return phi, ex


def _balance(s, prob, src, psi_in, phi, ex):
    q = s.quadrature()
    ang = s.tracks_angles()
    c = (2 * math.pi * q["w"][ang][:, None] * q["delta"][ang][:, None]
         * (q["w_polar"] * np.sqrt(1 - q["mu"] ** 2))[None, :])                   # [T, P]
    V = s.volumes()
    st = prob.sigma_t[prob.region_material]
    lhs = np.einsum("r,rg->g", V, st * phi - src)
    rhs = np.einsum("tp,tspg->g", c, psi_in - ex)
    scale = np.einsum("r,rg->g", V, st * np.abs(phi) + np.abs(src))
    return np.abs(lhs - rhs) / scale


def test_cfg2_full_size_sweep_vs_oracle(cuda):
    from oracle.oracle import Oracle
    log("[full size] 17x17 lattice, one FP32 sweep vs the oracle")
    prob = P.config(2)
    o = Oracle.from_problem(prob)
    s = moc.Solver(prob, precision="f32")
    rng = np.random.default_rng(3)
    src = rng.uniform(0.1, 2.0, size=(s.R, s.G))
    psi = rng.uniform(0, 1, size=s.psi_shape()).astype(np.float32).astype(np.float64)
    o.set_psi(psi)
    ref = o.sweep(src)
    phi, ex = _sweep(s, _dev(src, cuda), _dev(psi, cuda), cuda)
    phi = _host(phi)
    err = np.max(np.abs(phi - ref) / ref)
    log(f"  max rel err {err:.2e}")
    assert err < 1e-5
    np.testing.assert_allclose(_host(ex), o.get_exit_psi(), rtol=1e-5, atol=1e-6)


def test_cfg4_full_size_sweep_vs_oracle(cuda):
    """The 271-pin hexagon with 33 groups in full against one oracle sweep, element by
    element, for the instance the benchmark runs (group batches of 8: five batches with 7
    padding groups, P = 3) and for batches of 11 (three batches, no padding)."""
    import os
    import torch
    from oracle.oracle import Oracle
    log("[full size] 271-pin hexagon, 33 groups: one FP32 sweep vs the oracle")
    prob = P.config(4)
    th = max(1, min(16, os.cpu_count() or 1))
    o = Oracle.from_problem(prob, threads=th)
    o.set_threads(th)
    s = moc.Solver(prob, precision="f32")
    assert s.info["n_groups"] == 33
    rng = np.random.default_rng(4)
    src = rng.uniform(0.1, 2.0, size=(s.R, s.G))
    psi = rng.uniform(0, 1, size=s.psi_shape()).astype(np.float32).astype(np.float64)
    o.set_psi(psi)
    ref = o.sweep(src)
    ref_ex = o.get_exit_psi()
    for gb in (0, 11):
        if gb:
            del s
            torch.cuda.empty_cache()
            s = moc.Solver(prob, precision="f32", group_batch=gb)
        phi, ex = _sweep(s, _dev(src, cuda), _dev(psi, cuda), cuda)
        phi = _host(phi)
        err = np.max(np.abs(phi - ref) / ref)
        log(f"  group batch {gb or 'default'}: max rel err {err:.2e}")
        assert err < 1e-5
        np.testing.assert_allclose(_host(ex), ref_ex, rtol=1e-5, atol=1e-6)
        del ex
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("cfg", [3, 4])
def test_large_sweep_balance_and_fp64_agreement(cfg, cuda):
    import torch
    log(f"[full size] workload {cfg}: balance identity and FP32 vs FP64")
    prob = P.config(cfg)
    rng = np.random.default_rng(cfg)
    s32 = moc.Solver(prob, precision="f32")
    src = rng.uniform(0.1, 2.0, size=(s32.R, s32.G))
    psi = rng.uniform(0, 1, size=s32.psi_shape()).astype(np.float32).astype(np.float64)
    src_d, psi_d = _dev(src, cuda), _dev(psi, cuda)
    phi32, ex32 = _sweep(s32, src_d, psi_d, cuda)
    phi32, ex32 = _host(phi32), _host(ex32)
    bal = _balance(s32, prob, src, psi, phi32, ex32)
    log(f"  FP32 balance residual per group: max {bal.max():.2e}")
    assert bal.max() < 1e-5
    del s32
    torch.cuda.empty_cache()
    s64 = moc.Solver(prob, precision="f64")
    phi64, ex64 = _sweep(s64, src_d, psi_d, cuda)
    phi64, ex64 = _host(phi64), _host(ex64)
    bal64 = _balance(s64, prob, src, psi, phi64, ex64)
    log(f"  FP64 balance residual per group: max {bal64.max():.2e}")
    assert bal64.max() < 1e-12
    err = np.max(np.abs(phi32 - phi64) / phi64)
    log(f"  FP32 vs FP64 max rel err {err:.2e}")
    assert err < 1e-5
    del s64
    torch.cuda.empty_cache()
