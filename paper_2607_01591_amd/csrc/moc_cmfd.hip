// CMFD acceleration of the power iteration on a coarse mesh of cells (Sec. 2.2, Alg.
// MOCHFEM_CMFD, radial part): after each transport sweep the fine scalar flux is
// homogenised onto the coarse cells, the coarse-mesh eigenproblem is solved with the
// sweep's net surface currents, and the fine flux and the incoming boundary fluxes are
// rescaled by the ratio of new to homogenised coarse flux.
//
// Coarse equations (nonlinear diffusion form; the paper does not write them out):
//   sum_s J_s + Vc Sigma_t,c phi_c,g - Vc sum_g' Sigma_s,c,g'->g phi_c,g'
//       = (1/k) Vc chi_c,g sum_g' nuSigma_f,c,g' phi_c,g'
// with J across a surface from cell i to j closed as
//   J = -Dhat (phi_j - phi_i) - Dtilde (phi_j + phi_i),
//   Dhat = L 2 D_i D_j / (D_i h_j + D_j h_i), D = 1 / (3 Sigma_t,c),
// Dtilde set so the sweep's flux reproduces the sweep's current, and J = Dtilde_b phi_i
// on the domain boundary. Homogenisation is flux-volume weighted with the track volumes.
//
// Solver: inverse power iteration M y = (1/k) F x (Wielandt shift k_s = k (1 + shift) once
// k has settled), each linear solve by BiCGSTAB preconditioned with the inverse of every
// cell's G x G diagonal block. The whole coarse solve runs in one 1024-thread workgroup:
// the coarse problem is small (cells x groups unknowns) and the solver is a chain of
// dependent reductions, so one compute unit with workgroup barriers beats a chain of
// grid-wide launches. All arithmetic is FP64.
#include <cmath>

#include "moc_kernels.h"

namespace moc {

namespace {

constexpr int kSolveThreads = 1024;

// sum over the workgroup, returned to every thread
__device__ double wg_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += sh[i];
    return t;
}

// ---------------------------------------------------------------- homogenisation
// One workgroup per coarse cell. Thread (chunk, g) sums over every nch-th region of
// the cell; the chunk partial sums meet in LDS. Output row of the cell:
//   [0] Vc, [1] sum V F, then G each of V phi, V Sigma_t phi, V nuSigma_f phi, V chi F,
//   then G x G of V Sigma_s,g'->g phi_g' (from g', to g).
__global__ __launch_bounds__(256) void k_cmfd_homog(const double *__restrict__ phi, const double *__restrict__ V,
                                                    const int *__restrict__ mat, const double *__restrict__ sigt_m,
                                                    const double *__restrict__ sigs_m, const double *__restrict__ nsf_m,
                                                    const double *__restrict__ chi_m, const int64_t *__restrict__ reg_off,
                                                    const int *__restrict__ reg, double *__restrict__ hsum, int G, int nch) {
    extern __shared__ double sm[];
    const int c = blockIdx.x;
    const int W = G + 4;
    double *acc = sm;                              // [nch][G][W]
    double *accv = sm + (size_t)nch * G * W;       // [nch][2] V, V F
    const int t = threadIdx.x, g = t % G, ch = t / G;
    const bool active = ch < nch;
    const int64_t r0 = reg_off[c], r1 = reg_off[c + 1];
    if (active) {
        double a_phi = 0, a_st = 0, a_nsf = 0, a_chi = 0, a_v = 0, a_f = 0;
        double *as = acc + ((size_t)ch * G + g) * W + 4;
        for (int g2 = 0; g2 < G; ++g2) as[g2] = 0.0;
        for (int64_t i = r0 + ch; i < r1; i += nch) {
            const int r = reg[i];
            const int m = mat[r];
            const double v = V[r];
            const double *ph = phi + (int64_t)r * G;
            const double w = v * ph[g];
            double F = 0.0;
            for (int gp = 0; gp < G; ++gp) F += nsf_m[m * G + gp] * ph[gp];
            a_phi += w;
            a_st += sigt_m[m * G + g] * w;
            a_nsf += nsf_m[m * G + g] * w;
            a_chi += chi_m[m * G + g] * v * F;
            if (g == 0) {
                a_v += v;
                a_f += v * F;
            }
            const double *row = sigs_m + ((int64_t)m * G + g) * G;   // from g to every g2
            for (int g2 = 0; g2 < G; ++g2) as[g2] += row[g2] * w;
        }
        double *a4 = acc + ((size_t)ch * G + g) * W;
        a4[0] = a_phi;
        a4[1] = a_st;
        a4[2] = a_nsf;
        a4[3] = a_chi;
        if (g == 0) {
            accv[2 * ch] = a_v;
            accv[2 * ch + 1] = a_f;
        }
    }
    __syncthreads();
    const int HS = 2 + 4 * G + G * G;
    double *out = hsum + (int64_t)c * HS;
    for (int e = t; e < HS; e += blockDim.x) {
        double s = 0.0;
        if (e < 2) {
            for (int k = 0; k < nch; ++k) s += accv[2 * k + e];
        } else if (e < 2 + 4 * G) {
            const int q = (e - 2) / G, gg = (e - 2) - q * G;
            for (int k = 0; k < nch; ++k) s += acc[((size_t)k * G + gg) * W + q];
        } else {
            const int f = e - 2 - 4 * G, from = f / G, to = f - from * G;
            for (int k = 0; k < nch; ++k) s += acc[((size_t)k * G + from) * W + 4 + to];
        }
        out[e] = s;
    }
}

// ---------------------------------------------------------------- coarse solve
struct SolveArgs {
    const double *hsum;
    const double *tally;       // surface rows start at row n_real
    int n_real, Gp, C, G;
    const int64_t *adj_off;
    const int *adj_surf, *adj_nbr;
    const double *adj_sign, *adj_L, *adj_h, *adj_hn;
    double *Bs, *Binv, *Aoff, *phih, *Dc, *Ldiag, *fchi, *fnsf, *vec, *ratio, *stats, *scal;
    int *piv;
    double tol, shift;
    int max_outer, max_inner;
};

// vectors of vec: x (eigenvector), y (solve), r, rh, p, v, s, t, yp, zs
enum { kVx = 0, kVy, kVr, kVrh, kVp, kVv, kVs, kVt, kVyp, kVzs, kNumVec };

__device__ void build_blocks(const SolveArgs &a, double inv_ks) {
    const int C = a.C, G = a.G, HS = 2 + 4 * G + G * G;
    const int64_t N = (int64_t)C * G;
    for (int64_t i = threadIdx.x; i < N * G; i += blockDim.x) {
        const int c = int(i / ((int64_t)G * G));
        const int g = int((i / G) % G), gp = int(i % G);
        const double *h = a.hsum + (int64_t)c * HS;
        const double php = a.phih[(int64_t)c * G + gp];
        double v = php > 0 ? -h[2 + 4 * G + gp * G + g] / php : 0.0;   // - Vc Sigma_s,gp->g
        if (g == gp) {
            const double ph = a.phih[(int64_t)c * G + g];
            v += a.Ldiag[(int64_t)c * G + g] + (ph > 0 ? h[2 + G + g] / ph : 0.0);
        }
        v -= a.fchi[(int64_t)c * G + g] * a.fnsf[(int64_t)c * G + gp] * inv_ks;
        a.Bs[i] = v;
    }
    __syncthreads();
    // invert each cell's block (Gauss-Jordan, partial pivoting); one thread per cell
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        double *A = a.Bs + (int64_t)c * G * G;      // read-only copy is kept in Bs
        double *B = a.Binv + (int64_t)c * G * G;
        // work on B = A, then B <- A^-1 in place with a pivot record in the row order
        for (int e = 0; e < G * G; ++e) B[e] = A[e];
        int piv_ok = 1;
        for (int col = 0; col < G; ++col) {
            int pr = col;
            double best = fabs(B[col * G + col]);
            for (int r = col + 1; r < G; ++r)
                if (fabs(B[r * G + col]) > best) {
                    best = fabs(B[r * G + col]);
                    pr = r;
                }
            if (!(best > 0)) {
                piv_ok = 0;
                break;
            }
            // record the swap in the unused space by swapping rows of B only; the inverse
            // is recovered by swapping columns back at the end (standard in-place GJ)
            if (pr != col)
                for (int e = 0; e < G; ++e) {
                    const double tmp = B[col * G + e];
                    B[col * G + e] = B[pr * G + e];
                    B[pr * G + e] = tmp;
                }
            a.piv[(int64_t)c * G + col] = pr;   // pivot row of this column
            const double inv = 1.0 / B[col * G + col];
            B[col * G + col] = 1.0;
            for (int e = 0; e < G; ++e) B[col * G + e] *= inv;
            for (int r = 0; r < G; ++r) {
                if (r == col) continue;
                const double f = B[r * G + col];
                if (f == 0.0) continue;
                B[r * G + col] = 0.0;
                for (int e = 0; e < G; ++e) B[r * G + e] -= f * B[col * G + e];
            }
        }
        if (piv_ok) {
            for (int col = G - 1; col >= 0; --col) {
                const int pr = a.piv[(int64_t)c * G + col];
                if (pr != col)
                    for (int r = 0; r < G; ++r) {
                        const double tmp = B[r * G + col];
                        B[r * G + col] = B[r * G + pr];
                        B[r * G + pr] = tmp;
                    }
            }
        } else {
            // singular block: fall back to the inverse diagonal
            for (int e = 0; e < G * G; ++e) B[e] = 0.0;
            for (int g = 0; g < G; ++g) {
                const double d = A[g * G + g];
                B[g * G + g] = d != 0.0 ? 1.0 / d : 0.0;
            }
        }
    }
    __syncthreads();
}

// out = A x (shifted coarse operator)
__device__ void matvec(const SolveArgs &a, const double *x, double *out) {
    const int C = a.C, G = a.G;
    const int64_t N = (int64_t)C * G;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *B = a.Bs + ((int64_t)c * G + g) * G;
        const double *xc = x + (int64_t)c * G;
        double s = 0.0;
        for (int gp = 0; gp < G; ++gp) s += B[gp] * xc[gp];
        for (int64_t k = a.adj_off[c]; k < a.adj_off[c + 1]; ++k) {
            const int j = a.adj_nbr[k];
            if (j >= 0) s += a.Aoff[k * G + g] * x[(int64_t)j * G + g];
        }
        out[i] = s;
    }
    __syncthreads();
}

__device__ void precond(const SolveArgs &a, const double *x, double *out) {
    const int C = a.C, G = a.G;
    const int64_t N = (int64_t)C * G;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *B = a.Binv + ((int64_t)c * G + g) * G;
        const double *xc = x + (int64_t)c * G;
        double s = 0.0;
        for (int gp = 0; gp < G; ++gp) s += B[gp] * xc[gp];
        out[i] = s;
    }
    __syncthreads();
}

// (F x)_c,g = fchi_c,g sum_g' fnsf_c,g' x_c,g'; returns sum of F x, writes it to out if given
__device__ double apply_F(const SolveArgs &a, const double *x, double *out, double scale, double *sh) {
    const int C = a.C, G = a.G;
    const int64_t N = (int64_t)C * G;
    double tot = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *fn = a.fnsf + (int64_t)c * G;
        const double *xc = x + (int64_t)c * G;
        double f = 0.0;
        for (int gp = 0; gp < G; ++gp) f += fn[gp] * xc[gp];
        const double v = a.fchi[i] * f;
        if (out) out[i] = scale * v;
        tot += v;
    }
    const double s = wg_sum(tot, sh);
    __syncthreads();
    return s;
}

// BiCGSTAB (right block-Jacobi preconditioning) on A y = b, y holds the initial guess;
// stops at ||r|| <= rtol ||b||. Returns the iterations taken.
__device__ int bicgstab(const SolveArgs &a, const double *b, double rtol, int max_it, double *sh) {
    const int64_t N = (int64_t)a.C * a.G;
    double *V = a.vec;
    double *y = V + kVy * N, *r = V + kVr * N, *rh = V + kVrh * N, *p = V + kVp * N, *v = V + kVv * N;
    double *s = V + kVs * N, *t = V + kVt * N, *yp = V + kVyp * N, *zs = V + kVzs * N;
    matvec(a, y, t);
    double bb = 0.0, rr = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const double ri = b[i] - t[i];
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        bb += b[i] * b[i];
        rr += ri * ri;
    }
    bb = wg_sum(bb, sh);
    rr = wg_sum(rr, sh);
    const double stop = rtol * rtol * bb;
    if (rr <= stop) return 0;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    int it = 0;
    for (it = 1; it <= max_it; ++it) {
        double rn = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) rn += rh[i] * r[i];
        rn = wg_sum(rn, sh);
        if (rn == 0.0 || omega == 0.0) break;   // breakdown: keep the current y
        const double beta = (rn / rho) * (alpha / omega);
        rho = rn;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        __syncthreads();
        precond(a, p, yp);
        matvec(a, yp, v);
        double rv = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) rv += rh[i] * v[i];
        rv = wg_sum(rv, sh);
        if (rv == 0.0) break;
        alpha = rho / rv;
        double ss = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
            y[i] += alpha * yp[i];
            const double si = r[i] - alpha * v[i];
            s[i] = si;
            ss += si * si;
        }
        ss = wg_sum(ss, sh);
        if (ss <= stop) break;
        precond(a, s, zs);
        matvec(a, zs, t);
        double ts = 0.0, tt = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
            ts += t[i] * s[i];
            tt += t[i] * t[i];
        }
        ts = wg_sum(ts, sh);
        tt = wg_sum(tt, sh);
        omega = tt > 0.0 ? ts / tt : 0.0;
        rr = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
            y[i] += omega * zs[i];
            const double ri = s[i] - omega * t[i];
            r[i] = ri;
            rr += ri * ri;
        }
        rr = wg_sum(rr, sh);
        if (rr <= stop) break;
    }
    __syncthreads();
    return it;
}

__global__ __launch_bounds__(kSolveThreads) void k_cmfd_solve(SolveArgs a) {
    __shared__ double sh[kSolveThreads / 64];
    const int C = a.C, G = a.G, HS = 2 + 4 * G + G * G;
    const int64_t N = (int64_t)C * G;
    // homogenised flux, diffusion coefficients, fission operator factors
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *h = a.hsum + (int64_t)c * HS;
        const double Vc = h[0], Vphi = h[2 + g], Vst = h[2 + G + g];
        a.phih[i] = Vc > 0 ? Vphi / Vc : 0.0;
        a.Dc[i] = Vst > 0 ? Vphi / (3.0 * Vst) : 0.0;
        a.fchi[i] = h[1] > 0 ? h[2 + 3 * G + g] / h[1] : 0.0;
        a.fnsf[i] = (Vphi > 0 && Vc > 0) ? h[2 + 2 * G + g] / (Vphi / Vc) : 0.0;
    }
    __syncthreads();
    // surface coefficients: Dhat, Dtilde from the net currents; leakage diagonal
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double phc = a.phih[i], Di = a.Dc[i];
        double diag = 0.0;
        for (int64_t k = a.adj_off[c]; k < a.adj_off[c + 1]; ++k) {
            const int j = a.adj_nbr[k];
            const double J = a.adj_sign[k] * a.tally[((int64_t)a.n_real + a.adj_surf[k]) * a.Gp + g];   // out of c
            double off = 0.0;
            if (j < 0) {
                diag += phc > 0 ? J / phc : 0.0;
            } else {
                const double phj = a.phih[(int64_t)j * G + g], Dj = a.Dc[(int64_t)j * G + g];
                const double L = a.adj_L[k], hi = a.adj_h[k], hj = a.adj_hn[k];
                const double den = Di * hj + Dj * hi;
                const double dh = (L > 0 && den > 0) ? L * 2.0 * Di * Dj / den : 0.0;
                const double dt = (phj + phc) > 0 ? (-J - dh * (phj - phc)) / (phj + phc) : 0.0;
                diag += dh - dt;
                off = -dh - dt;
            }
            a.Aoff[k * G + g] = off;
        }
        a.Ldiag[i] = diag;
    }
    __syncthreads();

    double *V = a.vec;
    double *x = V + kVx * N, *y = V + kVy * N;
    double *b = a.ratio;   // right-hand side; the ratios are written only at the end
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) x[i] = a.phih[i];
    __syncthreads();
    double k = a.scal[kScalK];
    const double fs = apply_F(a, x, nullptr, 0.0, sh);
    // coarse accuracy follows the outer iteration: a coarse solve that stops at a fixed
    // tolerance hands back corrections of that size forever and the outer iteration
    // stalls short of its fixed point
    double tol = a.tol;
    const double res_prev = a.scal[kScalRes];
    if (res_prev > 0 && isfinite(res_prev)) tol = fmin(tol, fmax(1e-13, 1e-2 * res_prev));
    double inv_ks = 0.0;    // 0: unshifted
    bool shifted = false;
    int outer = 0, inner_total = 0;
    for (outer = 1; outer <= a.max_outer && fs > 0; ++outer) {
        if (outer == 1 || shifted) build_blocks(a, inv_ks);
        const double lam = 1.0 / k - inv_ks;
        // A y = lam F x from y = x
        apply_F(a, x, b, lam, sh);
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) y[i] = x[i];
        __syncthreads();
        inner_total += bicgstab(a, b, tol * 0.1, a.max_inner, sh);
        const double fy = apply_F(a, y, nullptr, 0.0, sh);
        if (!(fy > 0)) break;
        const double rho = fy / fs;
        const double knew = 1.0 / (inv_ks + lam / rho);
        double dx = 0.0, nx = 0.0;
        const double sc = fs / fy;
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
            const double yi = y[i] * sc;
            dx += (yi - x[i]) * (yi - x[i]);
            nx += yi * yi;
            x[i] = yi;
        }
        dx = wg_sum(dx, sh);
        nx = wg_sum(nx, sh);
        const double dk = fabs(knew - k) / knew;
        k = knew;
        if (dk < tol && dx <= tol * tol * nx) break;
        // Wielandt shift once k has settled well inside the shift margin
        if (!shifted && a.shift > 0 && dk < 1e-4) shifted = true;
        if (shifted) inv_ks = 1.0 / (k * (1.0 + a.shift));
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const double ph = a.phih[i];
        a.ratio[i] = ph > 0 ? x[i] / ph : 1.0;
    }
    if (threadIdx.x == 0) {
        a.scal[kScalKPrev] = a.scal[kScalK];
        if (fs > 0 && k > 0 && isfinite(k)) a.scal[kScalK] = k;
        a.stats[0] = outer > a.max_outer ? a.max_outer : outer;
        a.stats[1] = inner_total;
        a.stats[2] = k;
        a.stats[3] = tol;
    }
}

// phi *= ratio(cell of the region); incoming psi *= ratio(cell of the track's first region)
template <typename Real>
__global__ void k_cmfd_prolong(double *__restrict__ phi, Real *__restrict__ psi, const double *__restrict__ ratio,
                               const int *__restrict__ cell_of, const int *__restrict__ entry_cell, int R, int G, int Gp,
                               int P, int nslots) {
    const int64_t nphi = (int64_t)R * G, npsi = (int64_t)2 * P * Gp * nslots;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nphi + npsi; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nphi) {
            const int r = int(i / G), g = int(i - (int64_t)r * G);
            phi[i] *= ratio[(int64_t)cell_of[r] * G + g];
        } else {
            const int64_t j = i - nphi;
            const int slot = int(j % nslots);
            const int g = int((j / nslots) % Gp);
            const int s = int(j / ((int64_t)nslots * Gp * P));
            const int c = entry_cell[s * nslots + slot];
            if (c >= 0 && g < G) psi[j] = (Real)((double)psi[j] * ratio[(int64_t)c * G + g]);
        }
    }
}

}  // namespace

#define CMFD_CHECK_LAUNCH()                                                     \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) throw Error(MOC_EHIP, hipGetErrorString(e_));     \
    } while (0)

static int cmfd_homog_chunks(int G) {
    int nch = 256 / G;
    const int lds_cap = int(48 * 1024 / (sizeof(double) * (size_t)G * (G + 4) + 2 * sizeof(double)));
    if (nch > lds_cap) nch = lds_cap;
    return nch < 1 ? 1 : nch;
}

void launch_cmfd(const DevProblem &d, const DevCoarse &cd, double *phi, void *psi, hipStream_t s) {
    if (d.G > 255) throw Error(MOC_EINVAL, "cmfd: at most 255 groups");
    const int nch = cmfd_homog_chunks(d.G);
    const size_t lds = sizeof(double) * ((size_t)nch * d.G * (d.G + 4) + 2 * (size_t)nch);
    if (nch * d.G > 256 || lds > 64 * 1024) throw Error(MOC_EINVAL, "cmfd: too many groups for the homogenisation kernel");
    hipLaunchKernelGGL(k_cmfd_homog, dim3(cd.C), dim3(256), lds, s, phi, d.V, d.mat, d.sigt_m, d.sigs_m, d.nsf_m, d.chi_m,
                       cd.cell_reg_off, cd.cell_reg, cd.hsum, d.G, nch);
    CMFD_CHECK_LAUNCH();
    SolveArgs a{};
    a.hsum = cd.hsum;
    a.tally = d.tally;
    a.n_real = d.R;
    a.Gp = d.Gp;
    a.C = cd.C;
    a.G = d.G;
    a.adj_off = cd.adj_off;
    a.adj_surf = cd.adj_surf;
    a.adj_nbr = cd.adj_nbr;
    a.adj_sign = cd.adj_sign;
    a.adj_L = cd.adj_L;
    a.adj_h = cd.adj_h;
    a.adj_hn = cd.adj_hn;
    a.Bs = cd.Bs;
    a.Binv = cd.Binv;
    a.Aoff = cd.Aoff;
    a.phih = cd.phih;
    a.Dc = cd.Dc;
    a.Ldiag = cd.Ldiag;
    a.fchi = cd.fchi;
    a.fnsf = cd.fnsf;
    a.vec = cd.vec;
    a.ratio = cd.ratio;
    a.stats = cd.stats;
    a.piv = cd.piv;
    a.scal = d.scal;
    a.tol = cd.tol;
    a.shift = cd.shift;
    a.max_outer = cd.max_outer;
    a.max_inner = cd.max_inner;
    hipLaunchKernelGGL(k_cmfd_solve, dim3(1), dim3(kSolveThreads), 0, s, a);
    CMFD_CHECK_LAUNCH();
    const int64_t n = (int64_t)d.R * d.G + (int64_t)2 * d.P * d.Gp * d.nslots;
    int64_t grid = (n + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_cmfd_prolong<double>, dim3((int)grid), dim3(256), 0, s, phi, (double *)psi, cd.ratio, cd.cell_of,
                           cd.entry_cell, d.R, d.G, d.Gp, d.P, d.nslots);
    else
        hipLaunchKernelGGL(k_cmfd_prolong<float>, dim3((int)grid), dim3(256), 0, s, phi, (float *)psi, cd.ratio, cd.cell_of,
                           cd.entry_cell, d.R, d.G, d.Gp, d.P, d.nslots);
    CMFD_CHECK_LAUNCH();
}

}  // namespace moc
