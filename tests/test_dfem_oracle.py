"""Pins for the DFEM-SN oracle (linear discontinuous elements on triangles, discrete
ordinates). Expected values come from outside the oracle: a globally linear angular flux
is an exact solution of the discrete equations (it lies in the element space and is
continuous, so the upwind traces are exact), the per-sweep neutron balance of the
zeroth moment, the infinite-medium eigenvalue (dense eigen-decomposition), and agreement
with the planar MOC oracle (an independent discretisation) within discretisation error."""
import math

import numpy as np
import pytest

from oracle import sn_oracle as SN
from oracle.oracle import Oracle
from paper_2607_01591_amd import problems as P


def element_frames(prob):
    xy, tri = prob.xy, prob.tri
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area = 0.5 * ((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1]))
    c = (p0 + p1 + p2) / 3.0
    return area, c, np.sqrt(area)


def jittered_box(G=1, bc=(0, 0, 0, 0), n=5, seed=3, A=8, Pn=2, mats=None):
    rng = np.random.default_rng(seed)
    if G == 1:
        st, ss = np.array([[1.2], [0.5], [2.0]]), np.array([[[0.6]], [[0.2]], [[1.5]]])
        nsf, chi = np.array([[1.1], [0.0], [0.0]]), np.array([[1.0], [0.0], [0.0]])
    else:
        st, ss, nsf, chi = P.draw_xs(rng, 1, 2, G)
    p = P.box_problem(1.3, 0.9, n, n - 1, G=G, sigma_t=st, sigma_s=ss, nu_sigma_f=nsf, chi=chi, bc=bc,
                      n_azim=A, n_polar=Pn, spacing=0.1, jitter=0.12, seed=seed)
    if mats is not None:
        p.region_material = np.asarray(mats, np.int32)
    return p


@pytest.mark.parametrize("d", [0, 3, 5, 10, 13])
def test_linear_angular_flux_is_reproduced(d):
    """psi = a + b x + c y in every element, q = Omega . grad psi + Sigma_t psi (linear per
    element), exact inflow on the boundary: the DFEM solution equals psi to round-off."""
    prob = jittered_box(n=6, seed=d)
    o = SN.SNOracle(prob, n_azim=8, n_polar=2)
    rng = np.random.default_rng(100 + d)
    T = o.T
    st = rng.uniform(0.1, 3.0, T)
    a, b, c = rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
    mux, muy, _, _, _ = SN.directions(8, 2)
    area, cen, L = element_frames(prob)
    v0 = a + b * cen[:, 0] + c * cen[:, 1]
    exact = np.stack([v0, b * L, c * L], 1)
    q = np.stack([mux[d] * b + muy[d] * c + st * v0, st * b * L, st * c * L], 1)
    psi = o.sweep_linear(d, st, q, a, b, c)
    np.testing.assert_allclose(psi, exact, rtol=0, atol=1e-12 * np.abs(exact).max())


def test_mass_matrices_match_numerical_quadrature():
    """Element mass matrices int u_j u_i against scipy's adaptive quadrature over each
    triangle (a route independent of the oracle's edge-midpoint rule). The linear-solution
    pin cannot see them: they cancel from both sides for a linear solution."""
    import scipy.integrate
    prob = jittered_box(n=3, seed=9)
    o = SN.SNOracle(prob, n_azim=4, n_polar=1)
    geo = o.geometry()
    area, cen, L = element_frames(prob)
    for t in range(0, o.T, 3):
        p0, p1, p2 = (prob.xy[v] for v in prob.tri[t])
        def u(x, y):
            return np.array([1.0, (x - cen[t, 0]) / L[t], (y - cen[t, 1]) / L[t]])
        ref = np.zeros((3, 3))
        for j in range(3):
            for i in range(3):
                f = lambda tt, ss: (lambda x: u(*x)[j] * u(*x)[i])(p0 + ss * (p1 - p0) + tt * (p2 - p0)) * 2 * area[t]
                ref[j, i] = scipy.integrate.dblquad(f, 0, 1, 0, lambda ss: 1 - ss, epsabs=1e-14, epsrel=1e-12)[0]
        np.testing.assert_allclose(geo["mass"][t], ref, rtol=1e-10, atol=1e-14 * area[t])


def test_balance_identity_per_sweep():
    """Zeroth moment, summed over elements: interior upwind fluxes cancel, so
    sum_e area (Sigma_t phi_0 - s_0) = boundary inflow - boundary outflow, where inflow on
    reflective sides is the previous sweep's mirrored angular flux."""
    prob = jittered_box(G=3, bc=(1, 0, 1, 0), n=5, seed=4, mats=None)
    o = SN.SNOracle(prob, n_azim=8, n_polar=2)
    rng = np.random.default_rng(2)
    o.sweep(rng.uniform(0.1, 1.0, o.shape()))
    prev = o.get_psi()
    src = rng.uniform(0.1, 1.0, o.shape())
    src[..., 1:] = rng.uniform(-0.3, 0.3, src[..., 1:].shape)
    phi = o.sweep(src)
    psi = o.get_psi()
    area, cen, L = element_frames(prob)
    mat = prob.region_material[prob.tri_region]
    st = prob.sigma_t[mat]                                    # [T, G]
    lhs = np.einsum("t,tg->g", area, st * phi[..., 0] - src[..., 0])
    mux, muy, w, rx, ry = SN.directions(8, 2)
    x0, y0, x1, y1 = prob.box
    inflow, outflow = np.zeros(o.G), np.zeros(o.G)
    geo = o.geometry()
    for t in range(o.T):
        for k in range(3):
            if geo["nbr"][t, k] >= 0:
                continue
            pa, pb = prob.xy[prob.tri[t, k]], prob.xy[prob.tri[t, (k + 1) % 3]]
            tvec = pb - pa
            ln = float(np.hypot(*tvec))
            n = np.array([tvec[1], -tvec[0]]) / ln
            pm = 0.5 * (pa + pb)
            u = lambda p: np.array([1.0, (p[0] - cen[t, 0]) / L[t], (p[1] - cen[t, 1]) / L[t]])
            iu = ln / 6.0 * (u(pa) + 4 * u(pm) + u(pb))      # int_f u_i ds
            side = -1 - geo["nbr"][t, k]
            for d in range(o.nd):
                on = mux[d] * n[0] + muy[d] * n[1]
                if on > 0:
                    outflow += w[d] * on * psi[d, t] @ iu
                elif on < 0 and prob.bc[side] == P.BC_REFLECTIVE:
                    dm = rx[d] if side < 2 else ry[d]
                    inflow += w[d] * (-on) * prev[dm, t] @ iu
    np.testing.assert_allclose(lhs, inflow - outflow, rtol=0, atol=1e-12 * np.abs(lhs).max())
    assert inflow.max() > 1e-3 * np.abs(lhs).max()


def test_infinite_medium_eigenvalue():
    """One material, reflective box: the exact discrete fixed point is flat (zero slopes)
    with k = k-infinity."""
    prob = P.homogenize(jittered_box(G=4, bc=(1, 1, 1, 1), n=4, seed=7), 0)
    o = SN.SNOracle(prob, n_azim=8, n_polar=2)
    r = o.solve(tol=1e-12, max_iter=5000)
    assert r["converged"]
    st, ss, nsf, chi = prob.sigma_t[0], prob.sigma_s[0], prob.nu_sigma_f[0], prob.chi[0]
    kinf = max(abs(np.linalg.eigvals(np.linalg.solve(np.diag(st) - ss.T, np.outer(chi, nsf)))))
    assert abs(r["k"] - kinf) < 1e-9
    phi = r["phi"]
    np.testing.assert_allclose(phi[..., 0], np.broadcast_to(phi[0, :, 0], phi[..., 0].shape), rtol=1e-9)
    assert np.abs(phi[..., 1:]).max() < 1e-9 * phi[..., 0].max()


def test_close_to_planar_moc_on_the_pin_cell():
    """The same pin cell solved by DFEM-SN (linear elements) and by the planar MOC oracle
    (flat source, fine tracks): both discretise the same transport problem, so k and the
    region-averaged fluxes agree to the discretisation error (about 1 %; the angular
    quadratures differ too)."""
    prob = P.pin_cell_8region(seed=1, n_azim=16, n_polar=3, spacing=0.02)
    moc = Oracle.from_problem(prob).solve(tol=1e-9, max_iter=5000)
    o = SN.SNOracle(prob, n_azim=16, n_polar=3)
    r = o.solve(tol=1e-9, max_iter=5000)
    assert moc["converged"] and r["converged"]
    area, _, _ = element_frames(prob)
    R = prob.n_regions
    reg_area = np.bincount(prob.tri_region, weights=area, minlength=R)
    phi_r = np.stack([np.bincount(prob.tri_region, weights=area * r["phi"][:, g, 0], minlength=R) / reg_area
                      for g in range(prob.n_groups)], 1)
    # same normalisation: sum V nuSf phi = 1 with exact areas
    nsf = prob.nu_sigma_f[prob.region_material]
    phi_r /= np.sum(reg_area[:, None] * nsf * phi_r)
    ref = moc["phi"] / np.sum(reg_area[:, None] * nsf * moc["phi"])
    assert abs(r["k"] - moc["k"]) < 2e-3
    assert np.abs(phi_r / ref - 1).max() < 2e-2
