"""Plain FP64 numpy oracle of the diffusion HFEM coarse-mesh solver and its red-black
response-matrix iteration (Sec. 2.1.2, Eqs. HFEM_functional, HFEM_weak_form,
HFEM_flux_expansion, HFEM_current_expansion, HFEM_flux_response; Sec. 3.1 for the
preassembly / source update / red-black sweep / flux reconstruction split).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

What it computes, in the paper's order:

* Nodes are the bricks of a rectilinear grid (x, y, z edges); node e = (k ny + j) nx + i.
* Volume basis (Eq. HFEM_flux_expansion): products of Legendre polynomials
  u = sqrt((2a+1)(2b+1)(2c+1)) P_a(xi) P_b(eta) P_c(zeta) of total degree a + b + c <= Nv on
  the node's reference cube, orthogonal with (u_i, u_j)_e = V_e delta_ij (u_0 = 1, so
  phi_0 is the node average).
* Face basis (Eq. HFEM_current_expansion): on a face normal to axis d, products
  v = sqrt((2m+1)(2n+1)) P_m(s) P_n(t) of degree m + n <= Nf in the two other axes taken
  in increasing order, with <v_m, v_n>_f = A_f delta_mn. Faces of a node: x-, x+, y-, y+,
  z-, z+; face DoF index = face * (modes per face) + mode.
* Stationarity of Eq. HFEM_functional in phi gives, per node, A phi + M^T j = s with
  A_ij = (grad u_i, D grad u_j) + (u_i, Sigma_r u_j), M_(f m), i = <v_m, u_i>_f and
  s_i = (u_i, Q) (Eq. HFEM_weak_form); j holds the moments of the outward net current.
  Every integral is taken here by tensor Gauss-Legendre quadrature.
* With face flux moments chi = Lambda^-1 M phi (Lambda = face areas) and the partial
  currents J+- = chi / 4 +- j / 2, eliminating phi gives Eq. HFEM_flux_response:
  J+ = R J- + B s, R = (2 I + Y)^-1 (Y - 2 I), B = (2 I + Y)^-1 C, with C = Lambda^-1 M A^-1
  and Y = C M^T. The two inversions are those of the reaction matrix A and of 2 I + Y.
* Incoming currents: across an interior face J- is the neighbour's J+ on the same face
  (the face bases of the two nodes coincide); on a reflective side J- = J+; on a vacuum
  side J- = 0.
* Red-black iteration: node colour (i + j + k) mod 2; one iteration updates every red
  node's J+ from the current incoming currents, then every black node's.
* Flux reconstruction: phi = A^-1 (s - M^T (J+ - J-)).

Readings (the paper defers the derivation to its references):
* D_g = 1 / (3 Sigma_t,g) (no transport cross section in the data);
  Sigma_r,g = Sigma_t,g - Sigma_s,g->g.
* Emission moments Q_g,i = chi_g F_i / k + sum_{g' != g} Sigma_s,g'->g phi_g',i (+ external),
  F_i = sum_g nuSigma_f,g phi_g,i; the groups are solved together (Jacobi) from the
  previous outer iterate, with a fixed number of red-black iterations per outer
  iteration; the current state carries over between outer iterations.
* k update k_new = k sum_e V_e F_e,0(new) / sum_e V_e F_e,0(old); residual = relative
  V-weighted L2 change of the fission-rate shape (eigen) or of phi_0 (fixed source).

Array conventions: moments [N, G, Np]; partial currents [N, G, Nf_total].
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as _leg

BC_VACUUM, BC_REFLECTIVE = 0, 1


def volume_modes(nv: int):
    """(a, b, c) degree triples of the volume basis, by total degree, a then b descending."""
    out = []
    for n in range(nv + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def face_modes(nf: int):
    """(m, n) degree pairs of a face basis, by total degree, m descending."""
    out = []
    for t in range(nf + 1):
        for m in range(t, -1, -1):
            out.append((m, t - m))
    return out


def _pnorm(deg, x):
    """sqrt(2 deg + 1) P_deg(x) and its derivative."""
    c = np.zeros(deg + 1)
    c[deg] = math.sqrt(2 * deg + 1)
    return _leg.legval(x, c), _leg.legval(x, _leg.legder(c))


def node_integrals(h, nv, nf, nq=None):
    """Stiffness K_ij = (grad u_i, grad u_j), mass (u_i, u_j), face coupling
    M [6 Nfb, Np] and face areas Lambda [6 Nfb] of one brick with sides h = (hx, hy, hz),
    all by tensor Gauss-Legendre quadrature."""
    vm, fm = volume_modes(nv), face_modes(nf)
    Np, Nfb = len(vm), len(fm)
    nq = nq or (nv + 2)
    x, w = _leg.leggauss(nq)
    h = np.asarray(h, float)
    V = float(np.prod(h))
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * V / 8.0
    pts = (X, Y, Z)
    U = np.zeros((Np,) + X.shape)
    dU = np.zeros((3, Np) + X.shape)
    for i, deg in enumerate(vm):
        vals = [_pnorm(deg[d], pts[d]) for d in range(3)]
        U[i] = vals[0][0] * vals[1][0] * vals[2][0]
        for d in range(3):
            prod = np.ones_like(X)
            for e in range(3):
                prod = prod * (vals[e][1] * (2.0 / h[e]) if e == d else vals[e][0])
            dU[d, i] = prod
    K = np.zeros((Np, Np))
    Mass = np.zeros((Np, Np))
    for i in range(Np):
        for j in range(Np):
            K[i, j] = np.sum(W * sum(dU[d, i] * dU[d, j] for d in range(3)))
            Mass[i, j] = np.sum(W * U[i] * U[j])
    M = np.zeros((6 * Nfb, Np))
    Lam = np.zeros(6 * Nfb)
    S, T = np.meshgrid(x, x, indexing="ij")
    WF = w[:, None] * w[None, :]
    for d in range(3):
        tr = [e for e in range(3) if e != d]
        area = h[tr[0]] * h[tr[1]]
        for side in range(2):
            f = 2 * d + side
            coord = -1.0 if side == 0 else 1.0
            for m, (p, q) in enumerate(fm):
                v = _pnorm(p, S)[0] * _pnorm(q, T)[0]
                Lam[f * Nfb + m] = area
                for i, deg in enumerate(vm):
                    ui = _pnorm(deg[d], np.array(coord))[0] * _pnorm(deg[tr[0]], S)[0] * _pnorm(deg[tr[1]], T)[0]
                    M[f * Nfb + m, i] = np.sum(WF * v * ui) * area / 4.0
    return K, Mass, M, Lam


def node_matrices(h, D, sr, nv, nf):
    """Reaction matrix A = D K + Sigma_r Mass, face coupling M and face areas Lambda."""
    K, Mass, M, Lam = node_integrals(h, nv, nf)
    return D * K + sr * Mass, M, Lam


def response(A, M, Lam):
    """R, B of Eq. HFEM_flux_response plus A^-1 and P = A^-1 M^T (reconstruction)."""
    Ainv = np.linalg.inv(A)
    C = (M @ Ainv) / Lam[:, None]
    Y = C @ M.T
    I = np.eye(len(Lam))
    K = np.linalg.inv(2.0 * I + Y)
    return K @ (Y - 2.0 * I), K @ C, Ainv, Ainv @ M.T


class HFEMOracle:
    """Diffusion HFEM on a rectilinear brick grid with a red-black response-matrix sweep."""

    def __init__(self, x_edges, y_edges, z_edges, node_material, sigma_t, sigma_s, nu_sigma_f, chi,
                 bc=(1, 1, 1, 1, 1, 1), nv=2, nf=1, n_inner=2):
        self.edges = [np.asarray(e, float) for e in (x_edges, y_edges, z_edges)]
        self.nx, self.ny, self.nz = (len(e) - 1 for e in self.edges)
        self.N = self.nx * self.ny * self.nz
        self.mat = np.asarray(node_material, np.int64).reshape(self.N)
        self.st, self.ss = np.asarray(sigma_t, float), np.asarray(sigma_s, float)
        self.nsf, self.chi = np.asarray(nu_sigma_f, float), np.asarray(chi, float)
        self.G = self.st.shape[1]
        self.bc = tuple(int(b) for b in bc)
        self.nv, self.nf, self.n_inner = nv, nf, n_inner
        self.Np, self.Nfb = len(volume_modes(nv)), len(face_modes(nf))
        self.Nft = 6 * self.Nfb
        N, G = self.N, self.G
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        self.ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
        self.h = np.stack([np.diff(self.edges[d])[self.ijk[:, d]] for d in range(3)], axis=1)
        self.V = np.prod(self.h, axis=1)
        self.color = self.ijk.sum(axis=1) % 2
        # neighbour across each face (-1 on the domain boundary)
        self.nbr = -np.ones((N, 6), np.int64)
        dims = (self.nx, self.ny, self.nz)
        stride = (1, self.nx, self.nx * self.ny)
        for d in range(3):
            lo = self.ijk[:, d] > 0
            hi = self.ijk[:, d] < dims[d] - 1
            idx = np.arange(N)
            self.nbr[lo, 2 * d] = idx[lo] - stride[d]
            self.nbr[hi, 2 * d + 1] = idx[hi] + stride[d]
        # preassembly: per node and group
        self.R = np.zeros((N, G, self.Nft, self.Nft))
        self.B = np.zeros((N, G, self.Nft, self.Np))
        self.Ainv = np.zeros((N, G, self.Np, self.Np))
        self.P = np.zeros((N, G, self.Np, self.Nft))
        self.M = np.zeros((N, self.Nft, self.Np))
        self.Lam = np.zeros((N, self.Nft))
        cache = {}
        for e in range(N):
            key = tuple(self.h[e])
            if key not in cache:
                cache[key] = node_integrals(self.h[e], nv, nf)
            K, Mass, M, Lam = cache[key]
            m = self.mat[e]
            for g in range(G):
                D = 1.0 / (3.0 * self.st[m, g])
                sr = self.st[m, g] - self.ss[m, g, g]
                self.R[e, g], self.B[e, g], self.Ainv[e, g], self.P[e, g] = response(D * K + sr * Mass, M, Lam)
            self.M[e], self.Lam[e] = M, Lam
        self.qext = None
        self.reset()

    # ------------------------------------------------------------------ state
    def reset(self):
        self.jp = np.zeros((self.N, self.G, self.Nft))
        self.phi = np.zeros((self.N, self.G, self.Np))
        self.phi[..., 0] = 1.0
        self.k = 1.0

    def shape(self):
        return (self.N, self.G, self.Np)

    def incoming(self, jp=None):
        """J- [N, G, Nft] from the outgoing currents: neighbour's J+ on the shared face,
        own J+ on a reflective side, zero on a vacuum side."""
        jp = self.jp if jp is None else jp
        jm = np.zeros_like(jp)
        F = self.Nfb
        for f in range(6):
            sl = slice(f * F, (f + 1) * F)
            opp = slice((f ^ 1) * F, ((f ^ 1) + 1) * F)
            inner = self.nbr[:, f] >= 0
            jm[inner, :, sl] = jp[self.nbr[inner, f], :, opp]
            if self.bc[f] == BC_REFLECTIVE:
                jm[~inner, :, sl] = jp[~inner, :, sl]
        return jm

    # ------------------------------------------------------------------ one sweep
    def sweep(self, q):
        """Given emission moments q [N, G, Np] (per unit volume), run n_inner red-black
        iterations from the carried currents and return the reconstructed flux moments."""
        s = self.V[:, None, None] * np.asarray(q, float)
        bq = np.einsum("ngij,ngj->ngi", self.B, s)
        for _ in range(self.n_inner):
            for col in (0, 1):
                sel = self.color == col
                jm = self.incoming()
                self.jp[sel] = np.einsum("ngij,ngj->ngi", self.R[sel], jm[sel]) + bq[sel]
        net = self.jp - self.incoming()
        return np.einsum("ngij,ngj->ngi", self.Ainv, s) - np.einsum("ngij,ngj->ngi", self.P, net)

    # ------------------------------------------------------------------ sources
    def emission(self, phi, k):
        """Q_g,i = chi_g F_i / k + sum_{g' != g} Sigma_s,g'->g phi_g',i (+ external)."""
        m = self.mat
        F = np.einsum("ng,ngi->ni", self.nsf[m], phi)
        ss = self.ss[m].copy()
        idx = np.arange(self.G)
        ss[:, idx, idx] = 0.0
        q = np.einsum("nhg,nhi->ngi", ss, phi) + self.chi[m][:, :, None] * F[:, None, :] / k
        if self.qext is not None:
            q = q + self.qext
        return q

    def fission_rate(self, phi):
        return float(np.sum(self.V * np.einsum("ng,ng->n", self.nsf[self.mat], phi[..., 0])))

    def set_external_source(self, q):
        self.qext = None if q is None else np.asarray(q, float).reshape(self.shape())

    # ------------------------------------------------------------------ outer iteration
    def solve(self, tol=1e-8, max_iter=5000):
        """Outer iterations from a cold start (phi_0 = 1, currents 0, k = 1)."""
        self.reset()
        fixed = self.qext is not None
        it, res, dk = 0, np.inf, np.inf
        while it < max_iter:
            phi_old, k_old = self.phi, self.k
            new = self.sweep(self.emission(phi_old, k_old))
            it += 1
            if fixed:
                a = new[..., 0]
                b = phi_old[..., 0]
                res = math.sqrt(np.sum(self.V[:, None] * (a - b) ** 2) / max(np.sum(self.V[:, None] * a * a), 1e-300))
                dk = 0.0
                self.phi = new
            else:
                f_new, f_old = self.fission_rate(new), self.fission_rate(phi_old)
                self.k = k_old * f_new / f_old
                dk = abs(self.k - k_old)
                a = np.einsum("ng,ng->n", self.nsf[self.mat], new[..., 0]) / f_new
                b = np.einsum("ng,ng->n", self.nsf[self.mat], phi_old[..., 0]) / f_old
                res = math.sqrt(np.sum(self.V * (a - b) ** 2) / max(np.sum(self.V * a * a), 1e-300))
                self.phi = new
            if res < tol and dk < tol:
                return dict(k=self.k, phi=self.phi.copy(), iterations=it, residual=res, converged=True)
        return dict(k=self.k, phi=self.phi.copy(), iterations=it, residual=res, converged=False)

    def run_iterations(self, n):
        """Exactly n outer iterations from a cold start."""
        self.reset()
        fixed = self.qext is not None
        for _ in range(n):
            phi_old, k_old = self.phi, self.k
            new = self.sweep(self.emission(phi_old, k_old))
            if not fixed:
                self.k = k_old * self.fission_rate(new) / self.fission_rate(phi_old)
            self.phi = new
        return self.k, self.phi.copy()
