"""Pins for the CMFD oracle (coarse-mesh currents, coarse operator, accelerated
iteration). Each expected value comes from something the oracle does not contain: an
exact identity of the discretisation (coarse balance), a closed form (partial current of
an isotropic flux, the eigenvalue of a Toeplitz coarse operator, k-infinity from a dense
eigen-decomposition), or the unaccelerated power iteration, itself pinned elsewhere."""
import math

import numpy as np
import pytest

from oracle import cmfd_oracle as CM
from oracle.oracle import Oracle
from paper_2607_01591_amd import problems as P


def _coarse_sums(o, n, rc, T):
    """Per-cell tally sum, partial inflow and outflow from the oracle's currents."""
    off, nbr = o.coarse_adjacency()
    jp, jin = o.currents()
    Tc = np.zeros((n, o.G))
    np.add.at(Tc, rc, T)
    inflow, outflow = jin.copy(), np.zeros((n, o.G))
    for i in range(n):
        for s in range(off[i], off[i + 1]):
            outflow[i] += jp[s]
            if nbr[s] >= 0:
                inflow[nbr[s]] += jp[s]
    return Tc, inflow, outflow


def balance_cases():
    """The problems of the coarse-balance pin (also used by the mutant tests)."""
    return BALANCE_CASES


BALANCE_CASES = [
    ("lattice3x3_vacuum2", P.square_lattice(3, 3, seed=1, n_azim=16, spacing=0.05, bc=(1, 0, 1, 0)), (3, 3)),
    ("lattice_2x2_cells_of_4x4", P.square_lattice(4, 4, seed=6, n_azim=8, spacing=0.08, bc=(0, 0, 0, 0)), (2, 2)),
    ("box_unaligned_cells", P.box_problem(1.3, 0.9, 6, 5, G=2, sigma_t=[[1.0, 2.0]], jitter=0.1,
                                          bc=(0, 1, 0, 1), n_azim=12, spacing=0.04), (3, 2)),
    ("hex_small", P.hex_assembly(seed=5, rings=3, edge=0.25, G=4, spacing=0.05, n_azim=16), (4, 4)),
]


@pytest.mark.parametrize("name,prob,grid", BALANCE_CASES, ids=[c[0] for c in BALANCE_CASES])
def test_coarse_balance_identity(name, prob, grid):
    """Along every track the tallied increments telescope: summed over the regions of a
    coarse cell they equal the partial current into the cell minus the partial current
    out, for any source and any incoming boundary flux. A dropped crossing, a wrong
    weight or a crossing tallied with the wrong angular flux breaks this."""
    o = Oracle.from_problem(prob)
    n, rc = P.coarse_cells(prob, *grid)
    o.set_coarse(n, rc)
    rng = np.random.default_rng(3)
    o.set_psi(rng.random(o.psi_shape()))
    _, T = o.sweep(rng.random((o.R, o.G)) + 0.1, return_tally=True)
    Tc, inflow, outflow = _coarse_sums(o, n, rc, T)
    scale = np.abs(inflow).max()
    np.testing.assert_allclose(Tc, inflow - outflow, rtol=0, atol=1e-12 * scale)


def test_uniform_flux_currents_closed_form():
    """With an incoming flux equal to the flat source's psi = q / (4 pi Sigma_t) the
    angular flux is the same constant on every track, so (i) every interior net current
    vanishes to round-off and (ii) the partial current out of a whole side of length L is
    the isotropic value pi psi L, up to the quadrature error, which falls as the polar and
    azimuthal orders grow."""
    errs = []
    for A, Pn in [(8, 1), (16, 2), (64, 4)]:
        prob = P.box_problem(1.0, 0.7, 4, 3, G=1, sigma_t=[[0.8]], bc=(0, 0, 0, 0),
                             n_azim=A, n_polar=Pn, spacing=0.01)
        o = Oracle.from_problem(prob)
        n, rc = P.coarse_cells(prob, 2, 1)          # two cells, split at x = 0.5
        o.set_coarse(n, rc)
        psi0 = 0.37
        o.set_psi(np.full(o.psi_shape(), psi0))
        o.sweep(np.full((o.R, 1), 4 * math.pi * 0.8 * psi0))
        off, nbr = o.coarse_adjacency()
        jp, jin = o.currents()
        J = CM.net_currents(off, nbr, jp, jin)
        for i in range(n):
            for s in range(off[i], off[i + 1]):
                if nbr[s] >= 0:
                    assert abs(J[s, 0]) < 1e-13
        # total outflow through the boundary = pi psi * perimeter; inflow the same
        out_b = sum(jp[s, 0] for i in range(n) for s in range(off[i], off[i + 1]) if nbr[s] < 0)
        exact = math.pi * psi0 * 2 * (1.0 + 0.7)
        errs.append(abs(out_b - exact) / exact)
        assert abs(jin.sum() - out_b) < 1e-12 * exact
    assert errs[-1] < 2e-3 and errs[0] > errs[-1]


def test_coarse_operator_toeplitz_eigenvalue():
    """One group, a row of N identical cells with Dhat coupling and a boundary
    coefficient equal to Dhat: the loss operator is the Toeplitz tridiagonal matrix
    VSa + Dhat tridiag(-1, 2, -1), whose smallest eigenvalue is
    VSa + 2 Dhat (1 - cos(pi / (N + 1))); k = V nuSf / that."""
    N, h, St, Sa, nSf = 6, 1.5, 0.9, 0.3, 0.45
    D = 1.0 / (3 * St)
    dh = h * 2 * D * D / (D * h / 2 + D * h / 2)   # L = h, centroid-to-face = h / 2
    off = np.zeros(N + 1, np.int64)
    nbr, geom_surf = [], {}
    cen = np.array([[(i + 0.5) * h, 0.5 * h] for i in range(N)])
    for i in range(N):
        lst = ([i - 1] if i > 0 else [-1]) + ([i + 1] if i < N - 1 else [-1])
        lst = sorted(set(lst))
        nbr += lst
        off[i + 1] = off[i] + len(lst)
        if i < N - 1:
            mid = np.array([(i + 1) * h, 0.5 * h])
            geom_surf[(i, i + 1)] = (h, mid)
            geom_surf[(i + 1, i)] = (h, mid)
    nbr = np.array(nbr)
    phic = np.ones((N, 1))
    V = h * h
    hom = (np.full(N, V), phic, np.full((N, 1), St), np.full((N, 1, 1), St - Sa),
           np.full((N, 1), nSf), np.ones((N, 1)))
    # currents chosen so that Dtilde = 0 inside and Dtilde_b = Dhat on the ends
    J = np.zeros((len(nbr), 1))
    for i in range(N):
        for s in range(off[i], off[i + 1]):
            if nbr[s] < 0:
                J[s] = dh * phic[i, 0]
    M, F, dhat, dtil = CM.coarse_system(off, nbr, J, (cen, geom_surf), hom)
    assert np.allclose(dtil[nbr >= 0], 0) and np.allclose(dhat[nbr >= 0], dh)
    lam = V * Sa + 2 * dh * (1 - math.cos(math.pi / (N + 1)))
    phi, k, _ = CM.coarse_eigen(M, F, np.ones((N, 1)), 1.0)
    assert abs(k - V * nSf / lam) < 1e-12
    exact = np.sin(np.pi * np.arange(1, N + 1) / (N + 1))
    np.testing.assert_allclose(phi[:, 0] / phi[0, 0], exact / exact[0], rtol=1e-10)


def test_coarse_operator_infinite_medium_k_inf():
    """No net currents and flat flux: the coarse eigenproblem is the infinite-medium one,
    whose k is the dominant eigenvalue of (Sigma_t - Sigma_s^T)^-1 chi nuSigma_f^T (dense
    eigen-decomposition, an independent route). A transposed scattering matrix changes k
    for these asymmetric cross sections."""
    prob = P.config(1)
    G = prob.n_groups
    st, ss, nsf, chi = prob.sigma_t[0], prob.sigma_s[0], prob.nu_sigma_f[0], prob.chi[0]
    A = np.diag(st) - ss.T
    kinf = max(abs(np.linalg.eigvals(np.linalg.solve(A, np.outer(chi, nsf)))))
    n = 4
    off = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    nbr = np.array([-1, 1, -1, 0, -1, 3, -1, 2])
    J = np.zeros((len(nbr), G))
    cen = np.array([[0.5, 0.5], [1.5, 0.5], [2.5, 0.5], [3.5, 0.5]])
    surf = {(0, 1): (1.0, np.array([1.0, 0.5])), (1, 0): (1.0, np.array([1.0, 0.5])),
            (2, 3): (1.0, np.array([3.0, 0.5])), (3, 2): (1.0, np.array([3.0, 0.5]))}
    hom = (np.ones(n), np.ones((n, G)), np.tile(st, (n, 1)), np.tile(ss, (n, 1, 1)),
           np.tile(nsf, (n, 1)), np.tile(chi, (n, 1)))
    M, F, _, _ = CM.coarse_system(off, nbr, J, (cen, surf), hom)
    _, k, _ = CM.coarse_eigen(M, F, np.ones((n, G)), 1.0)
    assert abs(k - kinf) < 1e-11
    assert abs(kinf - max(abs(np.linalg.eigvals(np.linalg.solve(np.diag(st) - ss, np.outer(chi, nsf)))))) > 1e-3


def test_plain_loop_equals_c_oracle_solve():
    """The Python driver without a coarse mesh is the C oracle's power iteration."""
    prob = P.square_lattice(2, 2, seed=4, n_azim=8, spacing=0.08, bc=(1, 0, 1, 0))
    a = Oracle.from_problem(prob).solve(tol=1e-8, max_iter=2000)
    b = CM.solve(Oracle.from_problem(prob), prob, tol=1e-8, max_iter=2000)
    assert a["iterations"] == b["iterations"]
    assert abs(a["k"] - b["k"]) < 1e-14
    np.testing.assert_allclose(b["phi"], a["phi"], rtol=1e-12)


@pytest.mark.parametrize("bc", [(1, 0, 1, 0), (1, 1, 1, 1)])
def test_cmfd_reaches_the_power_iteration_fixed_point_faster(bc):
    """The CMFD update is consistent: at the MOC fixed point the coarse problem returns
    the homogenised flux itself, so the accelerated iteration converges to the same k and
    flux as the plain power iteration, in fewer sweeps."""
    prob = P.square_lattice(4, 4, seed=8, n_azim=16, spacing=0.05, bc=bc)
    n, rc = P.coarse_cells(prob, 4, 4)
    plain = Oracle.from_problem(prob).solve(tol=1e-10, max_iter=5000)
    acc = CM.solve(Oracle.from_problem(prob), prob, tol=1e-10, max_iter=5000, n_cells=n, region_cell=rc)
    assert plain["converged"] and acc["converged"]
    assert abs(acc["k"] - plain["k"]) < 1e-8
    np.testing.assert_allclose(acc["phi"], plain["phi"], rtol=2e-7)
    assert acc["iterations"] * 2 < plain["iterations"]
