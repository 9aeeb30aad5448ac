"""Pins for the FP64 oracle: it is checked against mathematics it does not contain.

Each test names what fixes the expected value: a library routine for a textbook special
case, a closed form, an exact identity of the discretisation, an independent numerical
integral, or brute force on a tiny input. A plausible mistake in the oracle (a wrong
sign, a dropped term, a transposed scattering matrix, a wrong tally weight or volume,
a wrong link) fails at least one of them; ``test_oracle_mutants.py`` plants such
mistakes to show it.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.oracle import Oracle, layout, polar_gl
from paper_2607_01591_amd import problems as P


# ---------------------------------------------------------------- quadratures / laydown
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_polar_gl_matches_library_and_moments(n):
    mu, w = polar_gl(n)
    x, wl = np.polynomial.legendre.leggauss(2 * n)
    pos = x > 0
    order = np.argsort(-x[pos])
    np.testing.assert_allclose(mu, x[pos][order], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, wl[pos][order], rtol=0, atol=1e-14)
    # half-range moments of even powers are exact up to degree 4n - 2
    for k in range(0, 4 * n - 1, 2):
        assert abs(np.sum(w * mu ** k) - 1.0 / (k + 1)) < 1e-13


@pytest.mark.parametrize("W,H,A,d", [(1.26, 1.26, 16, 0.05), (21.42, 21.42, 64, 0.02),
                                     (3.0, 1.7, 32, 0.03), (30.0, 27.5, 64, 0.02)])
def test_layout_properties(W, H, A, d):
    phi, dl, nx, ny, wa = layout(W, H, A, d)
    assert np.all(np.diff(phi) > 0) and phi[0] > 0 and phi[-1] < math.pi
    np.testing.assert_allclose(phi + phi[::-1], math.pi, atol=1e-14)
    assert abs(wa.sum() - 1.0) < 1e-14
    assert np.all(dl <= d * (1 + 1e-12))
    # cyclic condition: the spacing projected on both sides is the same delta
    np.testing.assert_allclose((W / nx) * np.abs(np.sin(phi)), dl, rtol=1e-13)
    np.testing.assert_allclose((H / ny) * np.abs(np.cos(phi)), dl, rtol=1e-13)
    # each corrected angle stays within one nominal interval of its nominal angle
    nominal = 2 * math.pi * (np.arange(A // 2) + 0.5) / A
    assert np.all(np.abs(phi - nominal) < math.pi / A)


# ---------------------------------------------------------------- tracking
def _brute_segments(prob, x0, y0, ux, uy, L):
    """Independent tracker for tiny meshes: parameters where the line crosses any
    triangle edge, sorted; each interval's midpoint is located by a point-in-triangle
    test over all triangles; drop < 1e-12 then merge same-region runs."""
    xy, tri = prob.xy, prob.tri
    ts = {0.0, L}
    for e in range(len(tri)):
        for q in range(3):
            a, b = xy[tri[e, q]], xy[tri[e, (q + 1) % 3]]
            # solve x0 + s u = a + t (b - a)
            M = np.array([[ux, a[0] - b[0]], [uy, a[1] - b[1]]])
            det = np.linalg.det(M)
            if abs(det) < 1e-15:
                continue
            s, t = np.linalg.solve(M, np.array([a[0] - x0, a[1] - y0]))
            if -1e-12 <= t <= 1 + 1e-12 and 0 < s < L:
                ts.add(float(s))
    ts = sorted(ts)
    out = []
    for s0, s1 in zip(ts[:-1], ts[1:]):
        if s1 - s0 < 1e-12:
            continue
        m = 0.5 * (s0 + s1)
        px, py = x0 + m * ux, y0 + m * uy
        reg = None
        for e in range(len(tri)):
            A_, B_, C_ = xy[tri[e]]
            d1 = (B_[0] - A_[0]) * (py - A_[1]) - (B_[1] - A_[1]) * (px - A_[0])
            d2 = (C_[0] - B_[0]) * (py - B_[1]) - (C_[1] - B_[1]) * (px - B_[0])
            d3 = (A_[0] - C_[0]) * (py - C_[1]) - (A_[1] - C_[1]) * (px - C_[0])
            if d1 >= 0 and d2 >= 0 and d3 >= 0:
                reg = prob.tri_region[e]
                break
        assert reg is not None
        if out and out[-1][0] == reg:
            out[-1][1] += s1 - s0
        else:
            out.append([reg, s1 - s0])
    return out


@pytest.mark.parametrize("prob", [P.config(1), P.square_lattice(2, 1, seed=7, n_azim=8, spacing=0.2)],
                         ids=["pincell", "lattice2x1"])
def test_tracking_matches_brute_force(prob):
    o = Oracle.from_problem(prob)
    tr = o.tracks()
    ang = o.angles()
    reg, ln = o.segments()
    rng = np.random.default_rng(0)
    for t in rng.choice(o.T, size=min(o.T, 25), replace=False):
        ph = ang["phi"][tr["angle"][t]]
        x0, y0 = tr["xy"][t, :2]
        ref = _brute_segments(prob, x0, y0, math.cos(ph), math.sin(ph), tr["length"][t])
        a, b = tr["offset"][t], tr["offset"][t + 1]
        assert [r for r, _ in ref] == list(reg[a:b])
        np.testing.assert_allclose([l for _, l in ref], ln[a:b], rtol=0, atol=1e-11)


@pytest.mark.parametrize("cfg", [1, 2])
def test_chords_volumes_links(cfg):
    prob = P.config(cfg)
    o = Oracle.from_problem(prob)
    tr = o.tracks()
    reg, ln = o.segments()
    W, H = prob.box[2], prob.box[3]
    assert o.max_gap < 1e-9
    chord = np.add.reduceat(ln, tr["offset"][:-1])
    np.testing.assert_allclose(chord, tr["length"], rtol=0, atol=1e-11)
    # track ends lie on the box
    for k in (0, 2):
        x, y = tr["xy"][:, k], tr["xy"][:, k + 1]
        on = (np.abs(x) < 1e-9) | (np.abs(x - W) < 1e-9) | (np.abs(y) < 1e-9) | (np.abs(y - H) < 1e-9)
        assert on.all()
    V = o.volumes()
    assert abs(V.sum() - W * H) < 1e-12 * W * H
    assert (V > 0).all()
    # reflective box: the link table is a permutation of all track-senses
    link = tr["link"].ravel()
    assert (link >= 0).all()
    assert len(np.unique(link)) == link.size


def test_volumes_converge_to_areas():
    prob = P.config(1)
    A = prob.region_areas()
    errs = []
    for d in (0.05, 0.025, 0.0125, 0.00625):
        prob.spacing = d
        errs.append(np.abs(Oracle.from_problem(prob).volumes() - A).max() / A.max())
    assert errs[-1] < 0.25 * errs[0]
    assert errs[-1] < 2e-3


# ---------------------------------------------------------------- sweep closed forms
def test_pure_absorber_exit_flux():
    """Q = 0, vacuum, homogeneous: psi_out = psi_in exp(-Sigma_t L / sin theta)."""
    prob = P.box_problem(1.3, 0.9, 3, 2, sigma_t=[[0.7]], bc=(0, 0, 0, 0), n_azim=16,
                         n_polar=3, spacing=0.05, jitter=0.1, seed=3)
    o = Oracle.from_problem(prob)
    mu, _ = o.polar()
    sin_t = np.sqrt(1 - mu ** 2)
    tr = o.tracks()
    L = np.hypot(tr["xy"][:, 2] - tr["xy"][:, 0], tr["xy"][:, 3] - tr["xy"][:, 1])
    rng = np.random.default_rng(1)
    psi_in = rng.uniform(0.5, 2.0, size=o.psi_shape())
    o.set_psi(psi_in)
    o.sweep(np.zeros((o.R, 1)))
    out = o.get_exit_psi()
    expect = psi_in * np.exp(-0.7 * L[:, None, None, None] / sin_t[None, None, :, None])
    np.testing.assert_allclose(out, expect, rtol=1e-13)


def test_sweep_balance_identity():
    """Telescoping along every track: sum_r T_rg = sum_tracks,senses,p c_ap (psi_in - psi_out)
    for any source and incoming flux (checks that every increment is tallied once)."""
    prob = P.config(1)
    o = Oracle.from_problem(prob)
    rng = np.random.default_rng(5)
    psi_in = rng.uniform(0, 1, size=o.psi_shape())
    o.set_psi(psi_in)
    src = rng.uniform(0.1, 1.0, size=(o.R, o.G))
    phi, T = o.sweep(src, return_tally=True)
    out = o.get_exit_psi()
    ang = o.angles()
    mu, wp = o.polar()
    tr = o.tracks()
    a = tr["angle"]
    c = (2 * math.pi * ang["w"][a][:, None] * ang["delta"][a][:, None]
         * (wp * np.sqrt(1 - mu ** 2))[None, :])           # [T, P]
    rhs = np.einsum("tp,tspg->g", c, psi_in - out)
    np.testing.assert_allclose(T.sum(axis=0), rhs, rtol=1e-12, atol=1e-14)
    # reflective hand-off: the next incoming flux of each linked track-sense is the
    # exit flux of the track-sense that feeds it
    nxt = o.get_psi().reshape(o.T * 2, o.P, o.G)
    link = tr["link"].ravel()
    np.testing.assert_array_equal(nxt[link], out.reshape(o.T * 2, o.P, o.G))
    # and phi is consistent with the tally definition
    V = o.volumes()
    st = prob.sigma_t[prob.region_material]
    np.testing.assert_allclose(phi, src / st + T / (st * V[:, None]), rtol=1e-13)


def _exact_square_flux(a, sigt, Q):
    """Region-averaged scalar flux of a homogeneous pure-absorber square with a flat
    isotropic source and vacuum boundaries, by direct integration of the first-flight
    angular flux over area and direction (scipy quadrature; 8-fold azimuthal and
    2-fold polar symmetry, chord integral in closed form)."""
    def inner(theta, w):
        st = math.sin(theta)
        s, c = math.sin(w), math.cos(w)
        flat = a * (c - s) * (1 - math.exp(-sigt * a / (c * st)))
        if s > 0:
            kap = sigt / (s * c * st)
            ramp = a * s - (1 - math.exp(-kap * a * s)) / kap
        else:
            ramp = 0.0
        return st * st / sigt * (flat + 2 * ramp)
    J, _ = integrate.dblquad(inner, 0, math.pi / 4, 0, math.pi / 2, epsabs=1e-13, epsrel=1e-12)
    J *= 16
    return Q / sigt * (1 - J / (4 * math.pi * a * a))


def test_exact_integral_tiny_square():
    """MOC converges to the exact first-flight integral in each quadrature parameter:
    polar order, azimuthal count and track spacing, each refined with the others fine."""
    exact = _exact_square_flux(1.0, 1.0, 1.0)

    def err(A, Pn, d):
        prob = P.box_problem(1.0, 1.0, 2, 2, sigma_t=[[1.0]], one_region=True, bc=(0, 0, 0, 0),
                             n_azim=A, n_polar=Pn, spacing=d)
        return abs(Oracle.from_problem(prob).sweep(np.ones((1, 1)))[0, 0] - exact)

    e_p = [err(256, n, 0.001) for n in (2, 4, 8, 16)]
    e_a = [err(A, 32, 0.001) for A in (16, 32, 64, 128)]
    e_d = [err(256, 32, d) for d in (0.04, 0.02, 0.01)]
    for seq in (e_p, e_a, e_d):
        assert all(e1 < e0 / 2.5 for e0, e1 in zip(seq, seq[1:])), seq
    assert err(256, 32, 0.001) < 2e-5 * exact


# ---------------------------------------------------------------- whole solver
def _kinf(st, ss, nsf, chi):
    A = np.diag(st) - ss.T
    M = np.linalg.solve(A, np.outer(chi, nsf))
    w, v = np.linalg.eig(M)
    i = np.argmax(w.real)
    vec = np.abs(v[:, i].real)
    return w[i].real, vec


def test_infinite_medium_eigenvalue():
    base = P.config(1)
    prob = P.homogenize(base, 0)
    prob.n_azim, prob.spacing = 8, 0.1
    o = Oracle.from_problem(prob)
    r = o.solve(tol=1e-12, max_iter=5000)
    assert r["converged"]
    k, vec = _kinf(prob.sigma_t[0], prob.sigma_s[0], prob.nu_sigma_f[0], prob.chi[0])
    assert abs(r["k"] - k) < 1e-10
    phi = r["phi"]
    spec = phi[0] / phi[0].sum()
    np.testing.assert_allclose(spec, vec / vec.sum(), rtol=1e-9)
    np.testing.assert_allclose(phi, np.broadcast_to(phi[0], phi.shape), rtol=1e-9)


def test_fixed_source_q_over_sigma_a():
    prob = P.box_problem(1.0, 1.0, 3, 3, sigma_t=[[1.0]], sigma_s=[[[0.6]]], jitter=0.1,
                         n_azim=8, spacing=0.1, seed=2)
    o = Oracle.from_problem(prob)
    o.set_external_source(np.full((o.R, 1), 1.0))
    r = o.solve(tol=1e-12, max_iter=20000, eigen=False)
    assert r["converged"]
    np.testing.assert_allclose(r["phi"], 1.0 / 0.4, rtol=1e-10)


@pytest.fixture(scope="module")
def cfg1_solution():
    prob = P.config(1)
    o = Oracle.from_problem(prob)
    return prob, o, o.solve(tol=1e-11, max_iter=5000)


def test_pincell_symmetry(cfg1_solution):
    prob, o, r = cfg1_solution
    phi = r["phi"]
    for a, b in [(0, 1), (2, 3), (4, 5), (4, 6), (4, 7)]:
        np.testing.assert_allclose(phi[a], phi[b], rtol=1e-10)


def test_reflective_balance_at_convergence(cfg1_solution):
    """With reflective sides there is no leakage: k = sum V nuSf phi / sum V Sa phi."""
    prob, o, r = cfg1_solution
    V = o.volumes()
    m = prob.region_material
    sa = prob.sigma_t[m] - prob.sigma_s[m].sum(axis=2)
    num = np.sum(V[:, None] * prob.nu_sigma_f[m] * r["phi"])
    den = np.sum(V[:, None] * sa * r["phi"])
    assert abs(num / den - r["k"]) < 1e-9


def test_scheme_independence(cfg1_solution):
    prob, _, ref = cfg1_solution
    for gsb, gse in [(True, False), (False, True), (True, True)]:
        o = Oracle.from_problem(prob)
        o.set_options(gs_boundary=gsb, gs_energy=gse)
        r = o.solve(tol=1e-11, max_iter=5000)
        assert r["converged"]
        assert abs(r["k"] - ref["k"]) < 1e-9
        np.testing.assert_allclose(r["phi"], ref["phi"], rtol=1e-8)


def test_links_are_geometric_reflections():
    """Every reflective link joins an exit point to the start point of the mirrored
    direction (checked from track end points, independently of the link search)."""
    prob = P.square_lattice(2, 2, seed=3, n_azim=16, spacing=0.1, bc=(1, 0, 1, 0))
    o = Oracle.from_problem(prob)
    tr = o.tracks()
    phi = o.angles()["phi"][tr["angle"]]
    u = np.stack([np.cos(phi), np.sin(phi)], 1)
    W, H = prob.box[2], prob.box[3]
    n_linked = 0
    for t in range(o.T):
        for s in range(2):
            exit_pt = tr["xy"][t, 2:] if s == 0 else tr["xy"][t, :2]
            d = u[t] if s == 0 else -u[t]
            side = (0 if abs(exit_pt[0]) < 1e-9 else 1 if abs(exit_pt[0] - W) < 1e-9
                    else 2 if abs(exit_pt[1]) < 1e-9 else 3)
            dst = tr["link"][t, s]
            if prob.bc[side] == 0:
                assert dst == -1
                continue
            n_linked += 1
            t2, s2 = divmod(dst, 2)
            start = tr["xy"][t2, :2] if s2 == 0 else tr["xy"][t2, 2:]
            d2 = u[t2] if s2 == 0 else -u[t2]
            np.testing.assert_allclose(start, exit_pt, atol=1e-10)
            refl = np.array([-d[0], d[1]]) if side < 2 else np.array([d[0], -d[1]])
            np.testing.assert_allclose(d2, refl, atol=1e-12)
    assert n_linked > 0


# ---------------------------------------------------------------- threads
def test_threads_change_nothing_but_summation_order():
    """The threaded track loop and tracker (a timing convenience) give the serial answer:
    tracking is identical, one sweep's flux, exit flux and coarse currents agree to 1e-12,
    a short power iteration agrees to 1e-12, and one thread reproduces the serial sums."""
    prob = P.square_lattice(4, 3, seed=31, n_azim=32, spacing=0.03, bc=(1, 0, 1, 0))
    o1 = Oracle.from_problem(prob, threads=1)
    o4 = Oracle.from_problem(prob, threads=4)
    r1, l1 = o1.segments()
    r4, l4 = o4.segments()
    assert np.array_equal(r1, r4) and np.array_equal(l1, l4)
    assert np.array_equal(o1.volumes(), o4.volumes())
    assert o4.set_threads(4), "oracle built without OpenMP"
    rng = np.random.default_rng(5)
    src = rng.uniform(0.1, 2.0, size=(o1.R, o1.G))
    psi0 = rng.uniform(0.0, 1.0, size=o1.psi_shape())
    n_cells, cells = P.coarse_cells(prob, 4, 3)   # coarse currents too
    out = []
    for o in (o1, o4):
        o.set_coarse(n_cells, cells)
        o.set_psi(psi0)
        phi, T = o.sweep(src, return_tally=True)
        jp, jin = o.currents()
        out.append((phi, T, o.get_exit_psi(), o.get_psi(), jp, jin))
    for a, b in zip(*out):
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-14 * np.abs(a).max())
    # one thread: the very same sums as the serial loop (bit for bit)
    o4.set_threads(1)
    o4.set_psi(psi0)
    phi1, T1 = o4.sweep(src, return_tally=True)
    assert np.array_equal(phi1, out[0][0]) and np.array_equal(T1, out[0][1])
    # a short power iteration
    o1b = Oracle.from_problem(prob, threads=1)
    o4b = Oracle.from_problem(prob, threads=4)
    ra = o1b.solve(tol=1e-30, max_iter=25)
    rb = o4b.solve(tol=1e-30, max_iter=25)
    assert abs(ra["k"] - rb["k"]) < 1e-12
    np.testing.assert_allclose(rb["phi"], ra["phi"], rtol=1e-12)
