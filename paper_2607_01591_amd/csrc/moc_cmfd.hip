// CMFD acceleration of the power iteration on a coarse mesh of cells (Sec. 2.1.2, Alg.
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
// k has settled, then fixed for the step), each linear solve by BiCGSTAB preconditioned
// with the inverse of every cell's G x G diagonal block. The solver is a chain of
// dependent reductions, so it runs as one launch: small coarse problems in one
// 1024-thread workgroup (workgroup barriers), larger ones on a cooperative grid with its
// own grid-wide barrier (below), never as a chain of launches. All arithmetic is FP64.
#include <algorithm>
#include <cmath>
#include <string>

#include "moc_kernels.h"

namespace moc {

namespace {

constexpr int kSolveThreads = 1024;

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
    double *red;               // exchange area of the grid team (kCmfdRedDoubles)
    double tol, shift;
    int max_outer, max_inner;
    int max_deg;               // most surfaces of any cell
};

constexpr int kMaxGridBlocks = 256;
// k counts as settled for the Wielandt shift when the last power iteration moved it by
// less than kSettled (relative), or the coarse iteration by less than kSettledCoarse
constexpr double kSettled = 1e-4, kSettledCoarse = 1e-4;
constexpr int kGridThreads = 256;   // threads per block of the cooperative solve (512 measured the same)
constexpr int64_t kGridSolveMinUnknowns = 4096;

// sums of v[0..NV) over the block, returned to every thread of the block (same order in
// every block); sh holds kMaxSums x 16 doubles
constexpr int kMaxSums = 6;
template <int NV> __device__ void block_sum_all(double (&v)[NV], double *sh) {
    static_assert(NV <= kMaxSums, "too many sums");
#pragma unroll
    for (int j = 0; j < NV; ++j)
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_down(v[j], off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[j * 16 + w] = v[j];
    __syncthreads();
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i) t += sh[j * 16 + i];
        v[j] = t;
    }
}

// The solver runs either in one workgroup (Team = WG) or in a cooperative grid (Team =
// GridTeam, grid-wide barriers). Both give every thread the same reduced values, in the
// same summation order, so every thread takes the same branches.
struct WG {
    double *sh;
    __device__ int64_t tid() const { return threadIdx.x; }
    __device__ int64_t size() const { return blockDim.x; }
    __device__ bool leader() const { return threadIdx.x == 0; }
    __device__ void sync() const { __syncthreads(); }
    __device__ bool failed() const { return false; }
    static constexpr bool kRegRows = false;   // 1024 threads: too few registers per thread
    template <int NV> __device__ void sum(double (&v)[NV]) { block_sum_all(v, sh); }
};

// Grid-wide barrier and reduction without a shared counter. Every block owns two 128-byte
// lines in the exchange area (picked by the parity of its barrier count): at a barrier its
// thread 0 stores the block's partial sums and then, with release ordering at device
// scope, the count itself; thread i of every block waits for block i's line to reach the
// count, reads the partials after an acquire fence, and the block sums them in block
// order. Waiting on nb separate lines in parallel costs about one memory round trip
// whatever nb is, where a shared arrival counter serialises nb atomics (measured 0.3 us
// per block and barrier). Two lines suffice: a block can only rewrite a line after
// passing the next barrier, which every reader of the line's previous value has reached
// after reading it. The area is zeroed before every launch. Waits are bounded: a wait
// longer than 2 s raises the abort word, every block then skips all
// remaining waits, and the aborted blocks' coarse ratios are NaN, which the host's
// finiteness check on the iterate reports.
constexpr int kLine = 16;                 // doubles per exchange line
constexpr unsigned long long kWaitLimitTicks = 200000000ull;   // 2 s of the 100 MHz real-time clock

__device__ bool wait_count(const double *line, unsigned long long want, unsigned *abort_word) {
    const unsigned long long *cnt = reinterpret_cast<const unsigned long long *>(line);
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (unsigned n = 0;; ++n) {
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) return true;
        if ((n & 63) == 63) {
            if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
            if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitLimitTicks) {
                __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int kThreads> struct GridTeam {
    double *sh;          // LDS, kMaxSums x 16 doubles
    int *lds_abort;      // LDS flag: a wait of this block gave up
    double *red;         // exchange area (global): lines of [count, values...]
    unsigned long long count = 0;
    bool aborted = false;
    __device__ int64_t tid() const { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
    __device__ int64_t size() const { return (int64_t)gridDim.x * blockDim.x; }
    __device__ bool leader() const { return blockIdx.x == 0 && threadIdx.x == 0; }
    __device__ bool failed() const { return aborted; }
    static constexpr bool kRegRows = kThreads <= 512;   // 1024 threads: too few registers
    // v: this block's sums (the same in every thread); returns the grid's sums, added in
    // block order in every block
    template <int NV> __device__ void exchange(double (&v)[NV]) {
        static_assert(NV + 1 <= kLine, "exchange line too short");
        ++count;
        const int par = int(count & 1);
        unsigned *abort_word = reinterpret_cast<unsigned *>(red + (size_t)kMaxGridBlocks * 2 * kLine);
        if (threadIdx.x == 0 && !aborted) {
            double *mine = red + ((size_t)blockIdx.x * 2 + par) * kLine;
#pragma unroll
            for (int j = 0; j < NV; ++j) mine[1 + j] = v[j];
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(mine), count, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        double p[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) p[j] = 0.0;
        if ((int)threadIdx.x < (int)gridDim.x && !aborted) {
            const double *line = red + ((size_t)threadIdx.x * 2 + par) * kLine;
            if (wait_count(line, count, abort_word)) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
                for (int j = 0; j < NV; ++j) p[j] = line[1 + j];
            } else {
                *lds_abort = 1;
            }
        }
        // the block sums' workgroup barriers order the other threads after the waits and
        // the pollers' acquire fences (which invalidate the caches the block reads through)
        block_sum_all(p, sh);
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = p[j];
        if (*lds_abort) aborted = true;
    }
    // Thread 0's release (an L2 write-back, then the store) covers the block's writes
    // only once they have reached L2, and a workgroup barrier does not wait for
    // outstanding global stores: every wavefront therefore waits for its own memory
    // operations (s_waitcnt 0) before the barrier that precedes thread 0's store. (A full
    // agent-scope release fence in every thread would do the same with one L2 write-back
    // per wavefront, which measured 2 ms more per CMFD step.)
    __device__ void sync() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        double z[1] = {0.0};
        exchange(z);
    }
    template <int NV> __device__ void sum(double (&v)[NV]) {
        __builtin_amdgcn_s_waitcnt(0);
        block_sum_all(v, sh);   // its workgroup barriers precede thread 0's release
        exchange(v);
    }
};

template <typename Team> __device__ double team_sum(Team &T, double v) {
    double z[1] = {v};
    T.sum(z);
    return z[0];
}

// vectors of vec: x (eigenvector), y (solve), r (two), rh, p (two), v, t, yp, zs
enum { kVx = 0, kVy, kVr0, kVr1, kVrh, kVp0, kVp1, kVv, kVt, kVyp, kVzs, kNumVec };
static_assert(kNumVec == kCmfdVectors, "solver vector count");

template <typename Team> __device__ void build_blocks(Team &T, const SolveArgs &a, double inv_ks) {
    const int C = a.C, G = a.G, HS = 2 + 4 * G + G * G;
    const int64_t N = (int64_t)C * G;
    for (int64_t i = T.tid(); i < N * G; i += T.size()) {
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
    T.sync();
    // invert each cell's block (Gauss-Jordan with partial pivoting, row swaps undone as
    // column swaps in reverse order at the end); one thread per cell
    for (int64_t c = T.tid(); c < C; c += T.size()) {
        const double *A = a.Bs + c * G * G;
        double *B = a.Binv + c * G * G;
        int *piv = a.piv + c * G;
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
            if (pr != col)
                for (int e = 0; e < G; ++e) {
                    const double tmp = B[col * G + e];
                    B[col * G + e] = B[pr * G + e];
                    B[pr * G + e] = tmp;
                }
            piv[col] = pr;
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
                const int pr = piv[col];
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
                const double dd = A[g * G + g];
                B[g * G + g] = dd != 0.0 ? 1.0 / dd : 0.0;
            }
        }
    }
    T.sync();
}

// Row i of the shifted coarse operator and of the block-Jacobi preconditioner, in two
// forms: read from global memory at every use (any size), or held in registers for the
// whole linear solve by the thread that owns the row (every thread owns at most one row,
// at most kRegG groups and kRegDeg surfaces per cell). Both sum in the same order.
struct MemRows {
    __device__ void load(const SolveArgs &, int64_t) {}
    __device__ double apply(const SolveArgs &a, const double *x, int64_t i) const {
        const int G = a.G;
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *B = a.Bs + i * G;
        const double *xc = x + (int64_t)c * G;
        double s = 0.0;
        for (int gp = 0; gp < G; ++gp) s += B[gp] * xc[gp];
        for (int64_t k = a.adj_off[c]; k < a.adj_off[c + 1]; ++k) {
            const int j = a.adj_nbr[k];
            if (j >= 0) s += a.Aoff[k * G + g] * x[(int64_t)j * G + g];
        }
        return s;
    }
    // sum over the cell's groups g' of Binv(i, g') u(cell row of g')
    template <typename U> __device__ double precond(const SolveArgs &a, int64_t i, U u) const {
        const int G = a.G;
        const int64_t c0 = (i / G) * G;
        const double *K = a.Binv + i * G;
        double s = 0.0;
        for (int gp = 0; gp < G; ++gp) s += K[gp] * u(c0 + gp);
        return s;
    }
};

constexpr int kRegG = 16, kRegDeg = 8;
struct RegRows {
    double B[kRegG], K[kRegG], off[kRegDeg];
    int nbr[kRegDeg];       // neighbour's row (same group), -1: none
    int c0 = 0;
    int G = 0;
    __device__ void load(const SolveArgs &a, int64_t i) {
        G = a.G;
#pragma unroll
        for (int e = 0; e < kRegG; ++e) B[e] = K[e] = 0.0;
#pragma unroll
        for (int e = 0; e < kRegDeg; ++e) {
            off[e] = 0.0;
            nbr[e] = -1;
        }
        if (i >= (int64_t)a.C * G) return;
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        c0 = c * G;
#pragma unroll
        for (int e = 0; e < kRegG; ++e)
            if (e < G) {
                B[e] = a.Bs[i * G + e];
                K[e] = a.Binv[i * G + e];
            }
        const int64_t k0 = a.adj_off[c], k1 = a.adj_off[c + 1];
#pragma unroll
        for (int e = 0; e < kRegDeg; ++e)
            if (k0 + e < k1) {
                const int j = a.adj_nbr[k0 + e];
                if (j >= 0) {
                    nbr[e] = j * G + g;
                    off[e] = a.Aoff[(k0 + e) * G + g];
                }
            }
    }
    __device__ double apply(const SolveArgs &, const double *x, int64_t) const {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < kRegG; ++e)
            if (e < G) s += B[e] * x[c0 + e];
#pragma unroll
        for (int e = 0; e < kRegDeg; ++e)
            if (nbr[e] >= 0) s += off[e] * x[nbr[e]];
        return s;
    }
    template <typename U> __device__ double precond(const SolveArgs &, int64_t, U u) const {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < kRegG; ++e)
            if (e < G) s += K[e] * u(c0 + e);
        return s;
    }
};

// (F x)_c,g = fchi_c,g sum_g' fnsf_c,g' x_c,g'; returns sum of F x, writes scale F x if out
template <typename Team>
__device__ double apply_F(Team &T, const SolveArgs &a, const double *x, double *out, double scale) {
    const int G = a.G;
    const int64_t N = (int64_t)a.C * G;
    double tot = 0.0;
    for (int64_t i = T.tid(); i < N; i += T.size()) {
        const int c = int(i / G);
        const double *fn = a.fnsf + (int64_t)c * G;
        const double *xc = x + (int64_t)c * G;
        double f = 0.0;
        for (int gp = 0; gp < G; ++gp) f += fn[gp] * xc[gp];
        const double v = a.fchi[i] * f;
        if (out) out[i] = scale * v;
        tot += v;
    }
    return team_sum(T, tot);   // the reduction's barrier also publishes out
}

// BiCGSTAB (right block-Jacobi preconditioning) on A y = b, y holds the initial guess;
// stops at ||r|| <= rtol ||b||. Returns the iterations taken. Four grid barriers per
// iteration: (1) after p and K^-1 p, (2) the reduction (rh, v), (3) after zs = K^-1 s,
// (4) one reduction of (t, s), (t, t), (rh, s), (rh, t), (s, s), from which omega, the
// new residual's norm ||s - omega t||^2 = (s,s) - 2 omega (t,s) + omega^2 (t,t) and
// (rh, r) = (rh, s) - omega (rh, t) follow without a fifth one. The residual r_n+1 of a
// row is stored by its owner after barrier (4), so the next iteration's cell-wise steps
// (which read the rows of other threads) form r_n+1 = r_n - alpha v - omega t from the
// published r_n, v and t; r and p alternate between two buffers so that no value is
// overwritten while another thread may still read it.
template <typename Team, typename Rows>
__device__ int bicgstab(Team &T, const SolveArgs &a, const Rows &R, const double *b, double rtol, int max_it) {
    const int64_t N = (int64_t)a.C * a.G;
    double *V = a.vec;
    double *y = V + kVy * N, *rh = V + kVrh * N, *v = V + kVv * N;
    double *t = V + kVt * N, *yp = V + kVyp * N, *zs = V + kVzs * N;
    double *rs[2] = {V + kVr0 * N, V + kVr1 * N};
    double *ps[2] = {V + kVp0 * N, V + kVp1 * N};
    double s0[2] = {0.0, 0.0};   // (b, b), (r, r)
    for (int64_t i = T.tid(); i < N; i += T.size()) {
        const double ri = b[i] - R.apply(a, y, i);
        rs[0][i] = ri;
        rs[1][i] = ri;
        rh[i] = ri;
        ps[0][i] = 0.0;
        v[i] = 0.0;
        t[i] = 0.0;
        s0[0] += b[i] * b[i];
        s0[1] += ri * ri;
    }
    T.sum(s0);
    const double stop = rtol * rtol * s0[0];
    if (s0[1] <= stop) return 0;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    double rn = s0[1];                 // (rh, r) with rh = r
    double al_prev = 0.0, om_prev = 0.0;   // the update that turns rs[cur ^ 1] into r_n
    int cur = 1;                       // rs[cur] holds r_n (stored by the rows' owners)
    int it = 0;
    for (it = 1; it <= max_it; ++it) {
        if (rn == 0.0 || omega == 0.0) break;   // breakdown: keep the current y
        const double beta = (rn / rho) * (alpha / omega);
        rho = rn;
        // p_n = r_n + beta (p_n-1 - omega v), yp = K^-1 p_n, from the cell's published rows
        {
            const double *rp = rs[cur ^ 1], *pp = ps[(it - 1) & 1];
            double *pn = ps[it & 1];
            const double bt = it == 1 ? 0.0 : beta, om = omega, ap = al_prev, op = om_prev;
            auto pcell = [&](int64_t j) { return (rp[j] - ap * v[j] - op * t[j]) + bt * (pp[j] - om * v[j]); };
            for (int64_t i = T.tid(); i < N; i += T.size()) {
                yp[i] = R.precond(a, i, pcell);
                pn[i] = pcell(i);
            }
        }
        T.sync();
        double s1[1] = {0.0};   // (rh, v)
        for (int64_t i = T.tid(); i < N; i += T.size()) {
            const double vi = R.apply(a, yp, i);
            v[i] = vi;
            s1[0] += rh[i] * vi;
        }
        T.sum(s1);
        if (s1[0] == 0.0) break;
        alpha = rho / s1[0];
        // zs = K^-1 s, s = r_n - alpha v, from the cell's rows
        {
            const double *rc = rs[cur];
            const double al = alpha;
            auto scell = [&](int64_t j) { return rc[j] - al * v[j]; };
            for (int64_t i = T.tid(); i < N; i += T.size()) zs[i] = R.precond(a, i, scell);
        }
        T.sync();
        double s5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // (t,s) (t,t) (rh,s) (rh,t) (s,s)
        for (int64_t i = T.tid(); i < N; i += T.size()) {
            const double ti = R.apply(a, zs, i);
            t[i] = ti;
            const double si = rs[cur][i] - alpha * v[i];
            s5[0] += ti * si;
            s5[1] += ti * ti;
            s5[2] += rh[i] * si;
            s5[3] += rh[i] * ti;
            s5[4] += si * si;
        }
        T.sum(s5);
        if (s5[4] <= stop) {
            // s already small enough: y += alpha yp and stop
            for (int64_t i = T.tid(); i < N; i += T.size()) y[i] += alpha * yp[i];
            break;
        }
        omega = s5[1] > 0.0 ? s5[0] / s5[1] : 0.0;
        // r_n+1 = s - omega t into the other buffer (its r_n-1 was last read before
        // barrier (1) of this iteration)
        double *rn1 = rs[cur ^ 1];
        for (int64_t i = T.tid(); i < N; i += T.size()) {
            y[i] += alpha * yp[i] + omega * zs[i];
            rn1[i] = (rs[cur][i] - alpha * v[i]) - omega * t[i];
        }
        const double rr = fmax(0.0, s5[4] - 2.0 * omega * s5[0] + omega * omega * s5[1]);
        rn = s5[2] - omega * s5[3];
        al_prev = alpha;
        om_prev = omega;
        cur ^= 1;
        if (rr <= stop) break;
    }
    T.sync();
    return it;
}

template <typename Team> __device__ void coarse_solve(Team &T, const SolveArgs &a) {
    const int C = a.C, G = a.G, HS = 2 + 4 * G + G * G;
    const int64_t N = (int64_t)C * G;
    // homogenised flux, diffusion coefficients, fission operator factors
    for (int64_t i = T.tid(); i < N; i += T.size()) {
        const int c = int(i / G), g = int(i - (int64_t)c * G);
        const double *h = a.hsum + (int64_t)c * HS;
        const double Vc = h[0], Vphi = h[2 + g], Vst = h[2 + G + g];
        a.phih[i] = Vc > 0 ? Vphi / Vc : 0.0;
        a.Dc[i] = Vst > 0 ? Vphi / (3.0 * Vst) : 0.0;
        a.fchi[i] = h[1] > 0 ? h[2 + 3 * G + g] / h[1] : 0.0;
        a.fnsf[i] = (Vphi > 0 && Vc > 0) ? h[2 + 2 * G + g] / (Vphi / Vc) : 0.0;
    }
    T.sync();
    // surface coefficients: Dhat, Dtilde from the net currents; leakage diagonal
    for (int64_t i = T.tid(); i < N; i += T.size()) {
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
    double *V = a.vec;
    double *x = V + kVx * N, *y = V + kVy * N;
    double *b = a.ratio;   // right-hand side; the ratios are written only at the end
    for (int64_t i = T.tid(); i < N; i += T.size()) x[i] = a.phih[i];
    T.sync();
    double k = a.scal[kScalK];
    const double fs = apply_F(T, a, x, nullptr, 0.0);
    // coarse accuracy follows the outer iteration: a coarse solve that stops at a fixed
    // tolerance hands back corrections of that size forever and the outer iteration
    // stalls short of its fixed point
    double tol = a.tol;
    const double res_prev = a.scal[kScalRes];
    if (res_prev > 0 && isfinite(res_prev)) tol = fmin(tol, fmax(1e-13, 0.1 * res_prev));
    // Wielandt shift from the start once the outer iteration's k has settled (|dk| of the
    // last power iteration well inside the shift margin); otherwise after the first
    // coarse iterations have settled it
    const double dk_prev = a.scal[kScalDk];
    bool shifted = a.shift > 0 && isfinite(dk_prev) && dk_prev < kSettled * k;
    double inv_ks = shifted ? 1.0 / (k * (1.0 + a.shift)) : 0.0;    // 0: unshifted
    int outer = 0, inner_total = 0;
    double built = -1.0;   // inv_ks of the blocks in Bs / Binv
    // operator rows in registers when every thread owns at most one (the same choice in
    // every thread)
    const bool regs = T.size() >= N && N < (int64_t)1 << 31 && G <= kRegG && a.max_deg <= kRegDeg;
    for (outer = 1; outer <= a.max_outer && fs > 0; ++outer) {
        if (inv_ks != built) {
            build_blocks(T, a, inv_ks);
            built = inv_ks;
        }
        const double lam = 1.0 / k - inv_ks;
        // A y = lam F x from y = x
        for (int64_t i = T.tid(); i < N; i += T.size()) y[i] = x[i];
        apply_F(T, a, x, b, lam);
        if constexpr (Team::kRegRows) {
            if (regs) {
                RegRows R;
                R.load(a, T.tid());
                inner_total += bicgstab(T, a, R, b, tol * 0.1, a.max_inner);
            } else {
                inner_total += bicgstab(T, a, MemRows{}, b, tol * 0.1, a.max_inner);
            }
        } else {
            inner_total += bicgstab(T, a, MemRows{}, b, tol * 0.1, a.max_inner);
        }
        const double fy = apply_F(T, a, y, nullptr, 0.0);
        if (!(fy > 0)) break;
        const double rho = fy / fs;
        const double knew = 1.0 / (inv_ks + lam / rho);
        double d2[2] = {0.0, 0.0};   // ||x_new - x||^2, ||x_new||^2
        const double sc = fs / fy;
        for (int64_t i = T.tid(); i < N; i += T.size()) {
            const double yi = y[i] * sc;
            d2[0] += (yi - x[i]) * (yi - x[i]);
            d2[1] += yi * yi;
            x[i] = yi;
        }
        T.sum(d2);
        const double dx = d2[0], nx = d2[1];
        const double dk = fabs(knew - k) / knew;
        k = knew;
        if (dk < tol && dx <= tol * tol * nx) break;
        // Wielandt shift once k has settled well inside the shift margin; the shift then
        // stays fixed for the rest of the step (the blocks and their inverses are built
        // once per shift), which converges as fast as following k here
        if (!shifted && a.shift > 0 && dk < kSettledCoarse) {
            shifted = true;
            inv_ks = 1.0 / (k * (1.0 + a.shift));
        }
    }
    T.sync();
    for (int64_t i = T.tid(); i < N; i += T.size()) {
        const double ph = a.phih[i];
        a.ratio[i] = T.failed() ? __builtin_nan("") : (ph > 0 ? x[i] / ph : 1.0);
    }
    if (T.leader()) {
        a.scal[kScalKPrev] = a.scal[kScalK];
        if (fs > 0 && k > 0 && isfinite(k)) a.scal[kScalK] = k;
        a.stats[0] = outer > a.max_outer ? a.max_outer : outer;
        a.stats[1] = inner_total;
        a.stats[2] = k;
        a.stats[3] = tol;
    }
}

__global__ __launch_bounds__(kSolveThreads) void k_cmfd_solve(SolveArgs a) {
    __shared__ double sh[kMaxSums * 16];
    WG T{sh};
    coarse_solve(T, a);
}

// the same solve over a cooperative grid (launched with hipLaunchCooperativeKernel)
template <int kThreads> __global__ __launch_bounds__(kThreads) void k_cmfd_solve_grid(SolveArgs a) {
    __shared__ double sh[kMaxSums * 16];
    __shared__ int lds_abort;
    if (threadIdx.x == 0) lds_abort = 0;
    __syncthreads();
    GridTeam<kThreads> T{sh, &lds_abort, a.red};
    coarse_solve(T, a);
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
    a.red = cd.red;
    a.scal = d.scal;
    a.tol = cd.tol;
    a.shift = cd.shift;
    a.max_outer = cd.max_outer;
    a.max_inner = cd.max_inner;
    a.max_deg = cd.max_deg;
    // large coarse problems: the same solve spread over a cooperative grid (one block of
    // 256 threads per 256 unknowns, at most kMaxGridBlocks); small ones: one workgroup,
    // whose barriers are cheaper than grid-wide ones
    const int64_t N = (int64_t)cd.C * d.G;
    int nb = cd.blocks;
    if (nb == 0)
        nb = N > kGridSolveMinUnknowns ? (int)std::min<int64_t>(kMaxGridBlocks, (N + kGridThreads - 1) / kGridThreads) : 1;
    if (nb > 1 && !cd.grid_ok) throw Error(MOC_EINVAL, "cmfd: the device does not support cooperative launches");
    if (nb > 1) {
        launch_fill_f64(cd.red, kCmfdRedDoubles, 0.0, s);   // barrier counts start at 0
        void *args[] = {&a};
        const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_cmfd_solve_grid<kGridThreads>), dim3(nb),
                                                        dim3(kGridThreads), args, 0, s);
        if (e != hipSuccess) throw Error(MOC_EHIP, std::string("cmfd: cooperative launch failed: ") + hipGetErrorString(e));
    } else {
        hipLaunchKernelGGL(k_cmfd_solve, dim3(1), dim3(kSolveThreads), 0, s, a);
        CMFD_CHECK_LAUNCH();
    }
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
