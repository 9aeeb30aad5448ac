"""Coarse-mesh finite-difference (CMFD) acceleration of the power iteration: a plain,
slow FP64 reference written with numpy and scipy on top of the C oracle's sweep.

TEST INFRASTRUCTURE ONLY: used by the test suite (and nothing in the product package).

What it follows. The paper accelerates its planar MOC with CMFD: each outer iteration
runs MOC on the fine mesh, homogenises the fine solution onto a coarse mesh, solves the
coarse-mesh problem with the MOC currents on the radial coarse surfaces, and updates the
fine-mesh solution with the accelerated result (Sec. 2.1.2, Alg. MOCHFEM_CMFD). In 2D
there is no axial (HFEM) part. The paper does not write out the coarse equations; the
reading used here is the standard nonlinear-diffusion form of CMFD:

* homogenisation by flux-volume weighting of the sweep's scalar flux, with the
  track-estimated region volumes (so that coarse balance is exact);
* net current across a coarse surface from cell i to cell j closed as
  J = -Dhat (phi_j - phi_i) - Dtilde (phi_j + phi_i), with
  Dhat = L * 2 D_i D_j / (D_i h_j + D_j h_i), D = 1 / (3 Sigma_t,c), L the shared edge
  length, h the distance from a cell's centroid to the surface's midpoint, and Dtilde
  chosen so that the MOC flux and current satisfy the closure exactly;
* on the domain boundary Dhat = 0 and J = Dtilde_b phi_i (vacuum and reflective alike);
* the coarse eigenproblem M phi = (1/k) F phi is solved to round-off by power iteration
  with direct sparse solves;
* the fine scalar flux and each track's incoming boundary flux are multiplied by the
  ratio of new to homogenised coarse flux of the cell they belong to (the cell of the
  track's first region for boundary fluxes), k is taken from the coarse problem, and the
  result is normalised like the plain power iteration.

Every function is a direct transcription of these definitions, with no blocking or
reordering.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FOUR_PI = 4.0 * np.pi


def fine_xs(prob):
    """Per-region cross sections from the material map: st [R,G], ss [R,G,G] (from, to),
    nsf [R,G], chi [R,G]."""
    m = np.asarray(prob.region_material)
    return (prob.sigma_t[m], prob.sigma_s[m], prob.nu_sigma_f[m], prob.chi[m])


def emission(prob, phi, k, qext=None):
    """Emission density s = sum_g' Sigma_s,g'->g phi_g' + chi_g F / k (+ q) (Eq. MGNTE)."""
    st, ss, nsf, chi = fine_xs(prob)
    F = np.sum(nsf * phi, axis=1)
    s = np.einsum("rpg,rp->rg", ss, phi) + chi * (F / k)[:, None]
    return s if qext is None else s + qext


def coarse_geometry(prob, n_cells, region_cell):
    """Cell centroids [C,2] (area-weighted) and, for every pair of cells sharing mesh
    edges, the shared length and its length-weighted midpoint: dict (i, j) -> (L, mid)."""
    xy, tri = prob.xy, prob.tri
    tcell = np.asarray(region_cell)[prob.tri_region]
    a = 0.5 * np.abs((xy[tri[:, 1], 0] - xy[tri[:, 0], 0]) * (xy[tri[:, 2], 1] - xy[tri[:, 0], 1])
                     - (xy[tri[:, 2], 0] - xy[tri[:, 0], 0]) * (xy[tri[:, 1], 1] - xy[tri[:, 0], 1]))
    cen_t = xy[tri].mean(axis=1)
    area = np.bincount(tcell, weights=a, minlength=n_cells)
    cen = np.stack([np.bincount(tcell, weights=a * cen_t[:, 0], minlength=n_cells),
                    np.bincount(tcell, weights=a * cen_t[:, 1], minlength=n_cells)], axis=1) / area[:, None]
    edges = {}
    for t in range(len(tri)):
        for e in range(3):
            u, v = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            edges.setdefault((min(u, v), max(u, v)), []).append(t)
    surf = {}
    for (u, v), ts in edges.items():
        if len(ts) != 2:
            continue
        ci, cj = int(tcell[ts[0]]), int(tcell[ts[1]])
        if ci == cj:
            continue
        L = float(np.hypot(*(xy[u] - xy[v])))
        mid = 0.5 * (xy[u] + xy[v])
        for key in ((ci, cj), (cj, ci)):
            L0, m0 = surf.get(key, (0.0, np.zeros(2)))
            surf[key] = (L0 + L, m0 + L * mid)
    surf = {key: (L, m / L) for key, (L, m) in surf.items()}
    return cen, surf


def homogenize(prob, phi, V, n_cells, region_cell):
    """Flux-volume-weighted coarse quantities: Vc [C], phic, stc, nsfc, chic [C,G],
    ssc [C,G,G] (from, to)."""
    st, ss, nsf, chi = fine_xs(prob)
    rc = np.asarray(region_cell)
    G = phi.shape[1]
    Vc = np.bincount(rc, weights=V, minlength=n_cells)

    def csum(x):  # sum over the regions of each cell
        out = np.zeros((n_cells,) + x.shape[1:])
        np.add.at(out, rc, x)
        return out

    Vphi = csum(V[:, None] * phi)
    phic = Vphi / Vc[:, None]
    stc = csum(V[:, None] * st * phi) / Vphi
    nsfc = csum(V[:, None] * nsf * phi) / Vphi
    ssc = csum(V[:, None, None] * ss * phi[:, :, None]) / Vphi[:, :, None]
    F = np.sum(nsf * phi, axis=1)
    fis = csum(V * F)
    chic = np.zeros((n_cells, G))
    pos = fis > 0
    chic[pos] = csum(chi * (V * F)[:, None])[pos] / fis[pos, None]
    return Vc, phic, stc, ssc, nsfc, chic


def net_currents(off, nbr, jpart, jin):
    """Net current leaving each cell through each adjacency slot (cell i -> nbr[s]):
    the partial current out through the slot minus the partial current back in."""
    n_cells = len(off) - 1
    J = np.zeros_like(jpart)
    slot = {}
    for i in range(n_cells):
        for s in range(off[i], off[i + 1]):
            slot[(i, int(nbr[s]))] = s
    for i in range(n_cells):
        for s in range(off[i], off[i + 1]):
            j = int(nbr[s])
            back = jin[i] if j < 0 else jpart[slot[(j, i)]]
            J[s] = jpart[s] - back
    return J


def coarse_system(off, nbr, J, geom, hom, k_ref=None):
    """Sparse M (loss: leakage closure + removal - scattering) and F (chi nuSigma_f), both
    [C G, C G] with unknown (c, g) at c G + g, plus Dhat / Dtilde per slot."""
    Vc, phic, stc, ssc, nsfc, chic = hom
    cen, surf = geom
    n_cells, G = phic.shape
    D = 1.0 / (3.0 * stc)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r); cols.append(c); vals.append(v)

    dhat = np.zeros_like(J)
    dtil = np.zeros_like(J)
    for i in range(n_cells):
        for s in range(off[i], off[i + 1]):
            j = int(nbr[s])
            for g in range(G):
                if j < 0:
                    # boundary: J = Dtilde_b phi_i
                    dt = J[s, g] / phic[i, g]
                    dtil[s, g] = dt
                    add(i * G + g, i * G + g, dt)
                    continue
                if (i, j) in surf:
                    L, mid = surf[(i, j)]
                    hi = np.hypot(*(cen[i] - mid))
                    hj = np.hypot(*(cen[j] - mid))
                    dh = L * 2.0 * D[i, g] * D[j, g] / (D[i, g] * hj + D[j, g] * hi)
                else:
                    dh = 0.0        # cells that touch only at a corner
                dt = (-J[s, g] - dh * (phic[j, g] - phic[i, g])) / (phic[j, g] + phic[i, g])
                dhat[s, g], dtil[s, g] = dh, dt
                # J_ij = -dh (phi_j - phi_i) - dt (phi_j + phi_i)
                add(i * G + g, i * G + g, dh - dt)
                add(i * G + g, j * G + g, -dh - dt)
        for g in range(G):
            add(i * G + g, i * G + g, Vc[i] * stc[i, g])
            for gp in range(G):
                add(i * G + g, i * G + gp, -Vc[i] * ssc[i, gp, g])
    N = n_cells * G
    M = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    fr, fc, fv = [], [], []
    for i in range(n_cells):
        for g in range(G):
            for gp in range(G):
                fr.append(i * G + g); fc.append(i * G + gp); fv.append(Vc[i] * chic[i, g] * nsfc[i, gp])
    F = sp.csr_matrix((fv, (fr, fc)), shape=(N, N))
    return M, F, dhat, dtil


def coarse_eigen(M, F, phi0, k0, tol=1e-13, max_iter=100000):
    """Power iteration on M phi = (1/k) F phi with direct solves, from (phi0, k0), until
    k and phi stop changing to round-off."""
    lu = spla.splu(M.tocsc())
    phi = phi0.reshape(-1).copy()
    k = k0
    fs = np.sum(F @ phi)
    for it in range(1, max_iter + 1):
        new = lu.solve(F @ phi / k)
        fs_new = np.sum(F @ new)
        k_new = k * fs_new / fs
        new *= fs / fs_new           # keep the production of phi fixed
        dphi = np.linalg.norm(new - phi) / np.linalg.norm(new)
        phi, dk, k = new, abs(k_new - k), k_new
        if dk < tol and dphi < tol * 10:
            return phi.reshape(phi0.shape), k, it
    raise RuntimeError("coarse eigenproblem did not converge")


def entry_cells(o, region_cell):
    """Coarse cell of the first region each track-sense meets, [T, 2] (-1: no segments)."""
    reg, _ = o.segments()
    off = o.tracks()["offset"]
    out = np.full((o.T, 2), -1, np.int64)
    has = off[1:] > off[:-1]
    rc = np.asarray(region_cell)
    out[has, 0] = rc[reg[off[:-1][has]]]
    out[has, 1] = rc[reg[off[1:][has] - 1]]
    return out


def solve(o, prob, tol=1e-6, max_iter=10000, n_cells=0, region_cell=None, phi0=None, k0=1.0,
          history=False):
    """Power iteration (Jacobi in energy, as the C oracle's ``solve``) with, when a coarse
    mesh is given, one CMFD update after every sweep. Returns the same fields as the C
    oracle's solve, plus per-iteration records when ``history``."""
    R, G = o.R, o.G
    V = o.volumes()
    st, ss, nsf, chi = fine_xs(prob)
    phi = np.ones((R, G)) if phi0 is None else np.array(phi0, float).reshape(R, G)
    k = float(k0)
    cmfd = n_cells > 0
    if cmfd:
        o.set_coarse(n_cells, region_cell)
        geom = coarse_geometry(prob, n_cells, region_cell)
        ent = entry_cells(o, region_cell)
    fs = np.sum(V[:, None] * nsf * phi)
    phi /= fs
    o.set_psi(o.get_psi() / fs)
    hist = []
    res = dk = 1.0
    conv = False
    for it in range(1, max_iter + 1):
        half = o.sweep(emission(prob, phi, k))
        psi = o.get_psi()               # incoming fluxes for the next sweep
        rec = {}
        if cmfd:
            off, nbr = o.coarse_adjacency()
            jp, jin = o.currents()
            J = net_currents(off, nbr, jp, jin)
            hom = homogenize(prob, half, V, n_cells, region_cell)
            M, F, dhat, dtil = coarse_system(off, nbr, J, geom, hom)
            phic_new, knew, cit = coarse_eigen(M, F, hom[1], k)
            ratio = phic_new / hom[1]
            new = half * ratio[region_cell]
            rt = np.where(ent[:, :, None] >= 0, ratio[np.maximum(ent, 0)], 1.0)  # [T,2,G]
            psi = psi * rt[:, :, None, :]
            rec = dict(k_cmfd=knew, coarse_iterations=cit, ratio=ratio, currents=J)
        else:
            new = half
            knew = k * np.sum(V[:, None] * nsf * half)
        fs = np.sum(V[:, None] * nsf * new)
        new /= fs
        o.set_psi(psi / fs)
        res = float(np.sqrt(np.sum(V[:, None] * (new - phi) ** 2) / np.sum(V[:, None] * new ** 2)))
        dk = abs(knew - k)
        phi, k = new, knew
        if history:
            rec.update(k=k, residual=res, phi=phi.copy())
            hist.append(rec)
        if res < tol and dk < tol:
            conv = True
            break
    out = dict(phi=phi, k=k, iterations=it, residual=res, dk=dk, converged=conv)
    if history:
        out["history"] = hist
    return out
