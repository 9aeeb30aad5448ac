"""Pins of the diffusion HFEM oracle (oracle/hfem_oracle.py) against what the mathematics
fixes, independently of the oracle's own arithmetic:

* A piecewise-quadratic diffusion solution (reflective at one end, Marshak vacuum at the
  other) lies in the trial spaces, so the hybrid method must reproduce its moments to
  rounding; one group along each axis, and two groups coupled by down- and up-scatter.
* Node integrals against closed forms of Legendre integrals.
* Infinite-medium eigenvalue with reflective sides (7 groups, upscatter).
* The bare-box one-group eigenvalue converges under h- and p-refinement to the analytic
  value with Marshak conditions, k = nuSigma_f / (Sigma_a + D B^2), tan(B a) = 1 / (2 D B)
  per axis; an octant with reflective symmetry planes gives the full box's eigenvalue.
* The flat-source slab converges to the analytic cosh solution under h- and p-refinement.
* Global neutron balance at convergence with vacuum sides.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L
from scipy.optimize import brentq

from oracle import hfem_oracle as H

VAC, REF = H.BC_VACUUM, H.BC_REFLECTIVE


def _grid(axis, edges):
    """Edges along `axis`; one unit-free node of width 1 along the two others."""
    out = [np.array([0.0, 1.0]), np.array([0.0, 0.7]), np.array([0.0, 1.3])]
    out[axis] = np.asarray(edges, float)
    return out


def _exact_moments(fun, edges_xyz, nv):
    """Moments (1/V) int f u_i dV of fun(x, y, z) on every node, by 8-point quadrature."""
    x, w = L.leggauss(8)
    ex, ey, ez = edges_xyz
    modes = H.volume_modes(nv)
    out = []
    for k in range(len(ez) - 1):
        for j in range(len(ey) - 1):
            for i in range(len(ex) - 1):
                lo = np.array([ex[i], ey[j], ez[k]])
                hi = np.array([ex[i + 1], ey[j + 1], ez[k + 1]])
                X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
                W = w[:, None, None] * w[None, :, None] * w[None, None, :] / 8.0
                P = [lo[d] + (hi[d] - lo[d]) * (Q + 1) / 2 for d, Q in enumerate((X, Y, Z))]
                f = fun(*P)
                row = []
                for (a, b, c) in modes:
                    u = np.ones_like(X)
                    for deg, Q in zip((a, b, c), (X, Y, Z)):
                        cc = np.zeros(deg + 1)
                        cc[deg] = math.sqrt(2 * deg + 1)
                        u = u * L.legval(Q, cc)
                    row.append(np.sum(W * f * u))
                out.append(row)
    return np.array(out)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("nv,nf", [(2, 0), (2, 1), (3, 1), (4, 2)])
def test_quadratic_solution_is_reproduced(axis, nv, nf):
    """phi = c - a t^2 on t in [0, H] (reflective at 0, Marshak vacuum at H), one group."""
    st, ss = 0.9, 0.4
    D, sr = 1.0 / (3.0 * st), st - ss
    Ht, a = 3.0, 0.2
    c = a * Ht * Ht + 4.0 * D * a * Ht           # phi(H)/4 + D phi'(H)/2 = 0
    edges = [0.0, 0.8, 1.9, 3.0]
    ex = _grid(axis, edges)
    bc = [REF] * 6
    bc[2 * axis + 1] = VAC
    o = H.HFEMOracle(*ex, np.zeros(3, int), [[st]], [[[ss]]], [[0.0]], [[0.0]], bc=bc, nv=nv, nf=nf, n_inner=2)
    t = lambda x, y, z: (x, y, z)[axis]
    q = _exact_moments(lambda x, y, z: 2 * D * a + sr * (c - a * t(x, y, z) ** 2), ex, nv)
    phi = _exact_moments(lambda x, y, z: c - a * t(x, y, z) ** 2, ex, nv)
    o.set_external_source(q[:, None, :])
    r = o.solve(tol=1e-14, max_iter=20000)
    assert r["converged"]
    err = np.abs(r["phi"][:, 0, :] - phi).max() / c
    assert err < 1e-10, err


def test_two_group_quadratic_with_up_and_down_scatter():
    """Two groups, both quadratic along z; the sources carry the cross-group transfers,
    so a transposed scattering matrix or a dropped transfer breaks the reproduction."""
    st = np.array([0.8, 1.4])
    ss = np.array([[0.3, 0.25], [0.05, 0.9]])     # [from][to]
    D = 1.0 / (3.0 * st)
    sr = st - np.diag(ss)
    Ht = 2.5
    a = np.array([0.3, 0.1])
    c = a * Ht * Ht + 4.0 * D * a * Ht
    ex = _grid(2, [0.0, 0.6, 1.7, 2.5])
    phi_f = [lambda x, y, z, g=g: c[g] - a[g] * z ** 2 for g in range(2)]
    ext = []
    for g in range(2):
        o_ = 1 - g
        ext.append(lambda x, y, z, g=g, o_=o_: 2 * D[g] * a[g] + sr[g] * phi_f[g](x, y, z) - ss[o_, g] * phi_f[o_](x, y, z))
    q = np.stack([_exact_moments(f, ex, 2) for f in ext], axis=1)
    phi = np.stack([_exact_moments(f, ex, 2) for f in phi_f], axis=1)
    bc = [REF, REF, REF, REF, REF, VAC]
    o = H.HFEMOracle(*ex, np.zeros(3, int), st[None], ss[None], np.zeros((1, 2)), np.zeros((1, 2)), bc=bc, nv=2, nf=1)
    o.set_external_source(q)
    r = o.solve(tol=1e-14, max_iter=20000)
    assert r["converged"]
    assert np.abs(r["phi"] - phi).max() / c.max() < 1e-10


def test_node_integrals_closed_forms():
    """Mass = V I; stiffness of the x-linear mode = 12 V / hx^2 (|d/dx sqrt(3) xi|^2 = 12 / hx^2);
    face coupling of u_0 = face area, of the x-linear mode = +-sqrt(3) area on x faces."""
    h = (0.7, 1.1, 2.3)
    V = np.prod(h)
    K, Mass, M, Lam = H.node_integrals(h, 3, 1)
    vm = H.volume_modes(3)
    assert np.allclose(Mass, V * np.eye(len(vm)), atol=1e-13)
    for d in range(3):
        i = vm.index(tuple(1 if e == d else 0 for e in range(3)))
        assert K[i, i] == pytest.approx(12.0 * V / h[d] ** 2, rel=1e-13)
        i2 = vm.index(tuple(2 if e == d else 0 for e in range(3)))
        # (2 / h)^2 (V / 8) 4 int (d/dxi sqrt(5) P2)^2 dxi, with d/dxi sqrt(5) P2 = 3 sqrt(5) xi
        # and int_-1^1 45 xi^2 dxi = 30
        assert K[i2, i2] == pytest.approx(2.0 * V / h[d] ** 2 * 30.0, rel=1e-13)
        assert K[0, i] == pytest.approx(0.0, abs=1e-12)
    areas = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    Nfb = len(H.face_modes(1))
    for f in range(6):
        assert Lam[f * Nfb] == pytest.approx(areas[f // 2])
        assert M[f * Nfb, 0] == pytest.approx(areas[f // 2], rel=1e-13)
        ix = vm.index(tuple(1 if e == f // 2 else 0 for e in range(3)))
        assert M[f * Nfb, ix] == pytest.approx((1 if f % 2 else -1) * math.sqrt(3) * areas[f // 2], rel=1e-13)


def test_infinite_medium_eigenvalue():
    from paper_2607_01591_amd import problems as P
    rng = np.random.default_rng(11)
    st, ss, nsf, chi = P.draw_xs(rng, 1, 0, 7)
    o = H.HFEMOracle([0, 1.0, 2.2], [0, 1.5, 2.0], [0, 0.9, 2.0], np.zeros(8, int), st, ss, nsf, chi, nv=2, nf=1)
    r = o.solve(tol=1e-12, max_iter=5000)
    Lm = np.diag(st[0]) - ss[0].T
    k_inf = max(abs(np.linalg.eigvals(np.linalg.solve(Lm, np.outer(chi[0], nsf[0])))))
    assert r["converged"]
    assert r["k"] == pytest.approx(k_inf, rel=1e-10)
    # flat flux: every node equal, no higher moments
    assert np.abs(r["phi"][..., 1:]).max() < 1e-9 * np.abs(r["phi"][..., 0]).max()


def _marshak_k(st, ss, nsf, half_widths):
    D, sa = 1.0 / (3.0 * st), st - ss
    b2 = 0.0
    for a in half_widths:
        B = brentq(lambda B: math.tan(B * a) - 1.0 / (2.0 * D * B), 1e-9, math.pi / (2 * a) - 1e-12)
        b2 += B * B
    return nsf / (sa + D * b2)


def _bare_box(n, nv, nf, W=(4.0, 3.0, 5.0), octant=False):
    st, ss, nsf = 1.0, 0.7, 0.36
    if octant:
        edges = [np.linspace(0, w / 2, n + 1) for w in W]
        bc = [REF, VAC, REF, VAC, REF, VAC]
    else:
        edges = [np.linspace(0, w, 2 * n + 1) for w in W]
        bc = [VAC] * 6
    N = np.prod([len(e) - 1 for e in edges])
    o = H.HFEMOracle(*edges, np.zeros(N, int), [[st]], [[[ss]]], [[nsf]], [[1.0]], bc=bc, nv=nv, nf=nf, n_inner=4)
    return o.solve(tol=1e-12, max_iter=20000), _marshak_k(st, ss, nsf, [w / 2 for w in W])


def test_bare_box_eigenvalue_converges_to_marshak_diffusion():
    errs_h = []
    for n in (1, 2, 3):
        r, k = _bare_box(n, 1, 0, octant=True)
        assert r["converged"]
        errs_h.append(abs(r["k"] - k) / k)
    assert errs_h[0] > errs_h[1] > errs_h[2]
    # p-refinement with the face order raised along with the volume order (a face order
    # far below the volume order limits the accuracy)
    errs_p = []
    for nv, nf in ((1, 0), (2, 1), (3, 2), (4, 2)):
        r, k = _bare_box(1, nv, nf, octant=True)
        errs_p.append(abs(r["k"] - k) / k)
    assert all(errs_p[i] > errs_p[i + 1] for i in range(3)), errs_p
    assert errs_p[-1] < 2e-4, errs_p


def test_octant_with_reflective_planes_equals_full_box():
    r_oct, _ = _bare_box(2, 2, 1, octant=True)
    r_full, _ = _bare_box(2, 2, 1, octant=False)
    assert r_oct["k"] == pytest.approx(r_full["k"], rel=1e-10)


@pytest.mark.parametrize("axis", [0, 2])
def test_flat_source_slab_converges_to_cosh(axis):
    st, ss, q0 = 1.2, 0.8, 1.0
    D, sr = 1.0 / (3.0 * st), st - ss
    Lh = math.sqrt(D / sr)
    Ht = 3.0
    alpha = 1.0 / (math.cosh(Ht / Lh) + 2.0 * D / Lh * math.sinh(Ht / Lh))
    exact = lambda t: q0 / sr * (1.0 - alpha * np.cosh(t / Lh))

    def err(n, nv, nf):
        ex = _grid(axis, np.linspace(0, Ht, n + 1))
        bc = [REF] * 6
        bc[2 * axis + 1] = VAC
        o = H.HFEMOracle(*ex, np.zeros(n, int), [[st]], [[[ss]]], [[0.0]], [[0.0]], bc=bc, nv=nv, nf=nf)
        q = np.zeros((n, 1, o.Np))
        q[:, 0, 0] = q0
        o.set_external_source(q)
        r = o.solve(tol=1e-14, max_iter=50000)
        ref = _exact_moments(lambda x, y, z: exact((x, y, z)[axis]), ex, nv)
        return np.abs(r["phi"][:, 0, 0] - ref[:, 0]).max() / (q0 / sr)

    eh = [err(n, 2, 1) for n in (2, 4, 8)]
    assert eh[0] / eh[1] > 8 and eh[1] / eh[2] > 8, eh      # O(h^4) or better on averages
    ep = [err(2, nv, 1) for nv in (1, 2, 3, 4)]
    assert all(ep[i] > ep[i + 1] for i in range(3)), ep
    assert ep[-1] < 1e-6, ep


def test_global_balance_with_vacuum_sides():
    """Sum of V Sigma_r phi_0 + leakage (area-weighted J+ through vacuum faces) equals the
    source plus in-scatter at convergence."""
    rng = np.random.default_rng(5)
    st = rng.uniform(0.5, 1.5, (2, 2))
    ss = np.zeros((2, 2, 2))
    ss[:, 0, 0] = 0.2
    ss[:, 1, 1] = 0.3
    ss[:, 0, 1] = 0.1
    edges = [np.array([0, 0.7, 1.5, 2.0]), np.array([0, 1.0, 1.8]), np.array([0, 1.2, 2.1, 2.4])]
    mat = rng.integers(0, 2, 18)
    o = H.HFEMOracle(*edges, mat, st, ss, np.zeros((2, 2)), np.zeros((2, 2)), bc=(VAC, REF, VAC, VAC, REF, VAC),
                     nv=2, nf=1)
    q = np.zeros(o.shape())
    q[..., 0] = rng.uniform(0.2, 1.0, (18, 2))
    q[..., 1:] = rng.uniform(-0.1, 0.1, (18, 2, o.Np - 1))
    o.set_external_source(q)
    r = o.solve(tol=1e-14, max_iter=50000)
    assert r["converged"]
    phi0 = r["phi"][..., 0]
    Nfb = o.Nfb
    for g in range(2):
        absorb = np.sum(o.V * (st[mat, g] - ss[mat, g, g]) * phi0[:, g])
        src = np.sum(o.V * q[:, g, 0])
        if g == 1:
            src += np.sum(o.V * ss[mat, 0, 1] * phi0[:, 0])
        leak = 0.0
        for f in range(6):
            if o.bc[f] == VAC:
                out = o.nbr[:, f] < 0
                leak += np.sum(o.Lam[out, f * Nfb] * o.jp[out, g, f * Nfb])
        assert absorb + leak == pytest.approx(src, rel=1e-10)
