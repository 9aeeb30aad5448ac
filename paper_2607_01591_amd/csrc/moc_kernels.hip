// HIP kernels of libmoc for gfx950 (CDNA4): source update, transport sweep, scalar-flux
// finalisation, FP64 reductions for the eigenvalue and residual, boundary-flux layout
// conversions.
//
// Layouts (internal region order r, which is a locality order of the user's regions):
//   xsq          : Real [R][Gp][2] = (Sigma_t, qhat) pairs; Gp = G padded (multiple of 4),
//                  padded groups hold zeros
//   tally        : double [R][Gp]
//   phi          : double [R][G]
//   psi          : Real [2 senses][P][Gp][nslots], slot = batch * 64 + lane
//   segments     : per batch, [step][64 lanes] of {length, region}; shorter tracks are
//                  padded with zero-length steps
#include <cmath>
#include <cstdio>

#include "moc_expf.h"
#include "moc_kernels.h"
#include "moc_pack.h"

namespace moc {

static constexpr double kFourPi = 12.566370614359172953850573533118;

template <typename Real> struct SegOf;
template <> struct SegOf<float> { using type = SegF; };
template <> struct SegOf<double> { using type = SegD; };

// MOC_EXP_TABLE: linear interpolation of f(x) = (1 - e^-x)/x on a uniform grid held in
// LDS; F = tau f(tau). Beyond the table the hardware exponential is used.
struct ExpTable {
    static constexpr int kN = kExpTableN;
    static constexpr float kMax = kExpTableMax;
};

// LDS of one sweep workgroup: the window tally [cap][GB] (FP64, or 64-bit fixed point in
// the FP32 sweep; 8 bytes either way), the window's slot -> region table for the flush,
// the per-group inverse fixed-point scales, and the exponential table (FP32 table mode).
template <typename Real, int GB, int MODE> struct SweepLds {
    static constexpr int kScaleSlots = 16;   // >= GB
    static constexpr size_t tab(int cap) { return sizeof(double) * GB * (size_t)cap; }
    static constexpr size_t scale(int cap) { return (tab(cap) + sizeof(int) * (size_t)cap + 7) / 8 * 8; }
    static constexpr size_t lut(int cap) { return scale(cap) + sizeof(double) * kScaleSlots; }
    static constexpr size_t bytes(int cap) {
        return lut(cap) + (MODE == MOC_EXP_TABLE && sizeof(Real) == 4 ? sizeof(float) * ExpTable::kN : 0);
    }
};

template <int MODE> __device__ __forceinline__ float one_minus_exp_f(float tau, const float *lut) {
    if constexpr (MODE == MOC_EXP_TABLE) {
        const float x = tau * (ExpTable::kN / ExpTable::kMax);
        if (x < float(ExpTable::kN - 1)) {
            const int i = int(x);
            const float fr = x - float(i);
            const float a = lut[i], b = lut[i + 1];
            return tau * (a + fr * (b - a));
        }
        return 1.0f - __builtin_amdgcn_exp2f(-tau * 1.4426950408889634f);
    } else {
        return -expm1f(-tau);
    }
}

template <typename Real, int MODE> __device__ __forceinline__ Real one_minus_exp(Real tau, const float *lut) {
    if constexpr (sizeof(Real) == 8) {
        return -expm1(-tau);
    } else {
        return one_minus_exp_f<MODE>(tau, lut);
    }
}

// ---------------------------------------------------------------- sweep
// One wavefront = one batch of 64 adjacent parallel tracks of one angle, one sense and
// one group batch [g0, g0 + GB). Lane l walks track l; the lanes step together through
// the batch's tally windows (forward windows and steps in order for sense 0, both
// reversed for sense 1). Per segment and group the update is Eq. MOC_sol:
// psi_out = qhat + (psi_in - qhat) e^-tau with tau = Sigma_t l / sin(theta_p); the
// increment Delta = (psi - qhat)(1 - e^-tau) is summed over the polar angles with the
// weights c_ap = 2 pi w_a w_p delta_a sin(theta_p) in registers, then added to the
// window-local tally slot in LDS. At the end of each window every slot is flushed with
// one FP64 atomic per group (consecutive lanes hit consecutive groups of a region row).
//
// FP32 sweep: the LDS window sums are 64-bit fixed point, since an integer LDS add
// (ds_add_u64) costs well under half of an FP64 one on gfx950. Along a segment the new
// angular flux is a convex combination of the old one and qhat, so with
// A_g = max(|qhat|, |incoming psi|) over the whole problem (tally_bound, formed before
// the sweep) every |psi - qhat| <= 2 A_g and every per-step polar sum is bounded by
// B = 2 A_g sum_p c_ap. The wave's scale for group g is s = 2^(50 - E), 2^(E-1) <= B < 2^E:
// each step's sum is rounded to the nearest multiple of 1/s (one FP64 fused multiply-add
// with 1.5 2^52, which leaves round(sum s) in the low mantissa bits while |sum s| < 2^51)
// and added as an integer; a slot takes at most kMaxSlotVisits (4095) terms, each below
// 2^50, so its sum stays below 2^62. The rounding error of a term is <= 2^(-51) B, far
// below the FP32 rounding of the sum itself; the flush converts each slot to FP64 and
// multiplies by 1/s (exact).
//
// CUR: the stream also holds coarse-surface crossing entries (region field >= n_real,
// length +-1 for the surface orientation). Their tally row holds Sigma_t = 1e30 and
// qhat = 0, so the same update gives Delta = psi; the angular flux is kept (psi -= 0 *
// Delta) and c_ap psi is tallied with the sign of the crossing direction, which makes
// the surface's tally row the net current across it.
template <typename Real, int NP, int GB, int MODE, bool CUR>
__global__ __launch_bounds__(64) void k_sweep(SweepArgs args) {
    using Seg = typename SegOf<Real>::type;
    using Lds = SweepLds<Real, GB, MODE>;
    constexpr bool kFix = sizeof(Real) == 4;   // 64-bit fixed-point window sums
    extern __shared__ unsigned char smem[];
    // tally [cap][GB]: FP64 (ds_add_f64 is far faster than ds_add_f32 on gfx950), or, in
    // the FP32 sweep, 64-bit fixed point (ds_add_u64 faster again)
    double *tl = reinterpret_cast<double *>(smem);
    unsigned long long *tlu = reinterpret_cast<unsigned long long *>(smem);
    const int cap = args.cap;
    double *winv = reinterpret_cast<double *>(smem + Lds::scale(cap));   // [GB] 1 / s per group
    float *lut = reinterpret_cast<float *>(smem + Lds::lut(cap));
    if constexpr (MODE == MOC_EXP_TABLE && sizeof(Real) == 4) {
        for (int i = threadIdx.x; i < ExpTable::kN; i += 64) lut[i] = args.exp_table[i];
    }
    for (int i = threadIdx.x; i < GB * cap; i += 64) tl[i] = 0.0;
    __syncthreads();

    const int b = args.batch_of_block[blockIdx.x], sense = blockIdx.y, gb = blockIdx.z, lane = threadIdx.x;
    const int nslots = args.nslots;
    const int slot = b * 64 + lane;
    const int g0 = gb * GB;
    const int Gp = args.Gp;
    const int a = args.batch_angle[b];
    const Seg *__restrict__ segs = reinterpret_cast<const Seg *>(args.segs);
    const Real *__restrict__ psi_in = reinterpret_cast<const Real *>(args.psi_in);
    Real *__restrict__ psi_out = reinterpret_cast<Real *>(args.psi_out);
    const Real *__restrict__ coef = reinterpret_cast<const Real *>(args.coef);
    const Real *__restrict__ inv_sin = reinterpret_cast<const Real *>(args.inv_sin);
    double *__restrict__ tally = args.tally;

    // per polar angle: tally weight, and the factor turning Sigma_t l into the exponent
    // argument (tau = Sigma_t l / sin(theta), or x = -tau log2(e) for the POLY mode)
    constexpr bool kDiff = sizeof(Real) == 4 && MODE == MOC_EXP_DIFF;
    constexpr bool kX = sizeof(Real) == 4 && (MODE == MOC_EXP_POLY || kDiff);
    Real c[NP], is[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        c[p] = coef[a * NP + p];
        is[p] = kX ? Real(-1.4426950408889634) * inv_sin[p] : inv_sin[p];
        // Keep these wave-uniform constants in vector registers. Left in the scalar
        // registers their loads fill, their first use inside the step loop makes the
        // compiler wait on the counter that scalar loads share with LDS operations at
        // every step, which also waits for the previous step's LDS tally atomics.
        if constexpr (sizeof(Real) == 4) {
            asm volatile("v_mov_b32 %0, %1" : "=v"(c[p]) : "s"(c[p]));
            asm volatile("v_mov_b32 %0, %1" : "=v"(is[p]) : "s"(is[p]));
        } else {
            asm volatile("v_mov_b64 %0, %1" : "=v"(c[p]) : "s"(c[p]));
            asm volatile("v_mov_b64 %0, %1" : "=v"(is[p]) : "s"(is[p]));
        }
    }
    Real psi[NP][GB];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < GB; ++j) psi[p][j] = psi_in[(int64_t)((sense * NP + p) * Gp + g0 + j) * nslots + slot];
    // fixed-point scale s of each group for this wave (FP32 sweep)
    double fsc[GB];
    if constexpr (kFix) {
        float csum = 0.f;
#pragma unroll
        for (int p = 0; p < NP; ++p) csum += fabsf((float)c[p]);
#pragma unroll
        for (int j = 0; j < GB; ++j) {
            const double B = 2.0 * (double)__uint_as_float(args.tally_bound[g0 + j]) * (double)csum;
            const bool finite = B <= 1.0e300;   // false for inf and NaN
            int E = 0;
            if (B > 0.0 && finite) frexp(B, &E);   // B = m 2^E, 1/2 <= m < 1
            E = E < -900 ? -900 : E;
            fsc[j] = finite ? ldexp(1.0, 50 - E) : 0.0;
            // a non-finite flux or source makes the tallies of the affected group NaN
            if (threadIdx.x == j) winv[j] = finite ? ldexp(1.0, E - 50) : __builtin_nan("");
        }
    }

    // Sigma_t and qhat of a region's group batch. One code path per instantiation: a
    // runtime choice between load widths would join two paths right after the loads and
    // force a wait on them, which defeats the look-ahead below. Even group batches start
    // on a 16-byte boundary (Gp is a multiple of 4), so they take float4 loads.
    const Real *__restrict__ xsq = reinterpret_cast<const Real *>(args.xsq);
    auto load_xs = [&](uint32_t key, Real (&st)[GB], Real (&q)[GB]) {
        const Real *row = xsq + ((int64_t)(key >> kSlotBits) * Gp + g0) * 2;
        if constexpr (sizeof(Real) == 4 && GB % 2 == 0) {
            float4 v[GB / 2];
#pragma unroll
            for (int u = 0; u < GB / 2; ++u) v[u] = reinterpret_cast<const float4 *>(row)[u];
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                const float4 &w = v[j >> 1];
                st[j] = (j & 1) ? w.z : w.x;
                q[j] = (j & 1) ? w.w : w.y;
            }
        } else if constexpr (sizeof(Real) == 4) {
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                const float2 w = reinterpret_cast<const float2 *>(row)[j];
                st[j] = w.x;
                q[j] = w.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                const double2 w = reinterpret_cast<const double2 *>(row)[j];
                st[j] = w.x;
                q[j] = w.y;
            }
        }
    };

    int *tabl = reinterpret_cast<int *>(smem + Lds::tab(cap));   // slot -> region
    const int64_t w0 = args.batch_win[b], w1 = args.batch_win[b + 1];
    for (int64_t wi = 0; wi < w1 - w0; ++wi) {
        const int64_t w = sense ? w1 - 1 - wi : w0 + wi;
        const int n = args.win_nsteps[w];
        const Seg *__restrict__ ws = segs + args.win_entry_off[w];
        // the window's slot table, fetched now and staged in LDS for the flush
        const int ns = args.win_nslots[w];
        const int *__restrict__ tab = args.win_tab + args.win_tab_off[w];
        int tabv[kMaxSlots / 64];
#pragma unroll
        for (int u = 0; u < kMaxSlots / 64; ++u) tabv[u] = (u * 64 + lane < ns) ? tab[u * 64 + lane] : 0;
        auto step_of = [&](int i) { return (int64_t)(sense ? n - 1 - i : i) * 64 + lane; };
        auto clampi = [&](int i) { return i < n ? i : n - 1; };
        // one step: Eq. MOC_sol for every group of the batch and polar angle, polar-summed
        // increments into the window's LDS tally
        auto update = [&](const Seg &sg, const Real (&st)[GB], const Real (&q)[GB]) {
            Real len = sg.len;
            const int ts = int(sg.key & ((1u << kSlotBits) - 1));
            Real cw[NP], keep = Real(1);
#pragma unroll
            for (int p = 0; p < NP; ++p) cw[p] = c[p];
            if constexpr (CUR) {
                const bool cross = len != Real(0) && (sg.key >> kSlotBits) >= (uint32_t)args.n_real;
                const Real sgn = (len > Real(0)) == (sense == 0) ? Real(1) : Real(-1);
                keep = cross ? Real(0) : Real(1);
                len = cross ? Real(1) : len;
#pragma unroll
                for (int p = 0; p < NP; ++p) cw[p] = cross ? c[p] * sgn : c[p];
            }
            // length times the per-polar factor once per step; the exponent of each update
            // is then Sigma_t times that
            Real lp[NP], acc[GB];
#pragma unroll
            for (int p = 0; p < NP; ++p) lp[p] = len * is[p];
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                acc[j] = 0;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if constexpr (kDiff) {
                        // e = e^-tau from the hardware exponential; the increment
                        // t (1 - e) with t = psi - qhat is formed by one fused multiply-add
                        // (t - t e, a single rounding), so its only error beyond that
                        // rounding is the absolute error of e
                        const Real e = __builtin_amdgcn_exp2f(st[j] * lp[p]);
                        const Real t = psi[p][j] - q[j];
                        const Real d = __builtin_fmaf(-t, e, t);
                        if constexpr (CUR)
                            psi[p][j] -= keep * d;
                        else
                            psi[p][j] -= d;
                        acc[j] += cw[p] * d;
                        continue;
                    }
                    Real F;
                    if constexpr (kX)
                        F = one_minus_exp2_poly(st[j] * lp[p]);
                    else
                        F = one_minus_exp<Real, MODE>(st[j] * lp[p], lut);
                    const Real d = (psi[p][j] - q[j]) * F;
                    if constexpr (CUR)
                        psi[p][j] -= keep * d;
                    else
                        psi[p][j] -= d;
                    acc[j] += cw[p] * d;
                }
            }
            if (len > Real(0)) {   // padding steps add nothing
                if constexpr (kFix) {
                    // round(acc s) as a 64-bit integer: adding 1.5 2^52 leaves it in the
                    // low mantissa bits
                    unsigned long long *row = tlu + ts * GB;
#pragma unroll
                    for (int j = 0; j < GB; ++j) {
                        const double v = __builtin_fma((double)acc[j], fsc[j], 6755399441055744.0);
                        atomicAdd(&row[j], (unsigned long long)__double_as_longlong(v) - 0x4338000000000000ull);
                    }
                } else {
                    double *row = tl + ts * GB;
#pragma unroll
                    for (int j = 0; j < GB; ++j) atomicAdd(&row[j], (double)acc[j]);
                }
            }
        };
        if constexpr (sizeof(Real) == 4) {
            // software pipeline: segment entries four steps ahead and cross sections two
            // steps ahead are in flight while the current step computes; unrolled by four
            // so every ring slot is a fixed register set (no copies between steps), and the
            // block of four twice more, which halves the drains of the load counter that
            // the compiler places at the loop's back edge
            Seg sg[4];
            Real st[4][GB], q[4][GB];
#pragma unroll
            for (int u = 0; u < 4; ++u) sg[u] = ws[step_of(clampi(u))];
            load_xs(sg[0].key, st[0], q[0]);
            load_xs(sg[1].key, st[1], q[1]);
#pragma unroll 2
            for (int i = 0; i < n; i += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    load_xs(sg[(u + 2) & 3].key, st[(u + 2) & 3], q[(u + 2) & 3]);
                    if (i + u < n) update(sg[u], st[u], q[u]);
                    sg[u] = ws[step_of(clampi(i + u + 4))];
                }
            }
        } else {
            // FP64: a shallower pipeline (register budget): segment entries two steps and
            // cross sections one step ahead
            Seg s0 = ws[step_of(0)], s1 = ws[step_of(clampi(1))];
            Real st0[GB], q0[GB];
            load_xs(s0.key, st0, q0);
            for (int i = 0; i < n; ++i) {
                const Seg s2 = ws[step_of(clampi(i + 2))];
                Real st1[GB], q1[GB];
                load_xs(s1.key, st1, q1);
                update(s0, st0, q0);
                s0 = s1;
                s1 = s2;
#pragma unroll
                for (int j = 0; j < GB; ++j) {
                    st0[j] = st1[j];
                    q0[j] = q1[j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxSlots / 64; ++u)
            if (u * 64 + lane < ns) tabl[u * 64 + lane] = tabv[u];
        __syncthreads();
        // flush the window's slots: (slot, group) pairs, groups fastest
        for (int e = lane; e < ns * GB; e += 64) {
            const int sl = e / GB, j = e - sl * GB;
            if constexpr (kFix) {
                const long long iv = (long long)tlu[e];
                const double iw = winv[j];
                if (iv != 0 || iw != iw) {
                    unsafeAtomicAdd(&tally[(int64_t)tabl[sl] * Gp + g0 + j], (double)iv * iw);
                    tlu[e] = 0ull;
                }
            } else {
                const double v = tl[e];
                if (v != 0.0) {
                    unsafeAtomicAdd(&tally[(int64_t)tabl[sl] * Gp + g0 + j], v);
                    tl[e] = 0.0;
                }
            }
        }
        __syncthreads();
    }
    const int dst = args.link[sense * nslots + slot];
    if (dst >= 0) {
        const int s2 = dst / nslots, slot2 = dst - s2 * nslots;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int j = 0; j < GB; ++j) psi_out[(int64_t)((s2 * NP + p) * Gp + g0 + j) * nslots + slot2] = psi[p][j];
    }
    if (!args.fed[sense * nslots + slot]) {
        // an incoming slot that no link feeds (vacuum side) stays zero in the next buffer
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int j = 0; j < GB; ++j) psi_out[(int64_t)((sense * NP + p) * Gp + g0 + j) * nslots + slot] = Real(0);
    }
    if (args.exit_canon) {
        const int t = args.canon_of_slot[slot];
        if (t >= 0) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int j = 0; j < GB; ++j)
                    if (g0 + j < args.G)
                        args.exit_canon[(((int64_t)t * 2 + sense) * NP + p) * args.G + g0 + j] = (double)psi[p][j];
        }
    }
}

// ---------------------------------------------------------------- small kernels
template <typename T> __global__ void k_fill(T *__restrict__ p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename T> __global__ void k_scale(T *__restrict__ p, int64_t n, const double *__restrict__ f) {
    const T s = (T)(*f);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] *= s;
}

// qhat from a caller's emission density (user order): qhat = s / (4 pi Sigma_t)
template <typename Real>
__global__ void k_prep_user(const double *__restrict__ src_user, const int *__restrict__ user_of, const int *__restrict__ mat,
                            const double *__restrict__ sigt_m, Real *__restrict__ xsq, int R, int G, int Gp) {
    const int64_t n = (int64_t)R * Gp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = int(i / Gp), g = int(i - (int64_t)r * Gp);
        Real v = 0;
        if (g < G) v = (Real)(src_user[(int64_t)user_of[r] * G + g] / (kFourPi * sigt_m[mat[r] * G + g]));
        xsq[2 * i + 1] = v;
    }
}

// Source update (Eq. MGNTE, isotropic): s_g = sum_g' Sigma_s,g'->g phi_g' + chi_g F / k
// (+ external), F = sum_g nuSigma_f,g phi_g; qhat = s / (4 pi Sigma_t). FP64 arithmetic.
// One thread per (region, group), consecutive threads on consecutive groups of a region
// (the fission sum is formed by each of them): G-fold more parallelism than a thread per
// region, which matters for many groups. Region and group indices fit 32 bits (regions
// are below 2^23 by the packed segment key).
template <typename Real>
__global__ void k_source(const double *__restrict__ phi, const double *__restrict__ scal, const int *__restrict__ mat,
                         const double *__restrict__ sigt_m, const double *__restrict__ sigs_m,
                         const double *__restrict__ nsf_m, const double *__restrict__ chi_m,
                         const double *__restrict__ qext, Real *__restrict__ xsq, int R, int G, int Gp) {
    const double inv_k = 1.0 / scal[kScalK];
    const uint32_t n = (uint32_t)R * (uint32_t)G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t r = i / (uint32_t)G, g = i - r * (uint32_t)G;
        const int m = mat[r];
        const double *ph = phi + (int64_t)r * G;
        const double *col = sigs_m + (int64_t)m * G * G + g;
        const double *nsf = nsf_m + m * G;
        double F = 0.0, s = 0.0;
        for (int gp = 0; gp < G; ++gp) {
            const double f = ph[gp];
            F += nsf[gp] * f;
            s += col[(int64_t)gp * G] * f;
        }
        s += chi_m[m * G + g] * F * inv_k;
        if (qext) s += qext[i];
        xsq[((int64_t)r * Gp + g) * 2 + 1] = (Real)(s / (kFourPi * sigt_m[m * G + g]));
    }
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

// phi = 4 pi qhat + T / (Sigma_t V) (angular integration of segment averages; FP64);
// either to the internal phi with per-block partials of sum V F, or to a user buffer.
// One thread per (region, group); the partial sums run over (region, group) pairs.
template <typename Real>
__global__ void k_finalize(const Real *__restrict__ xsq, const double *__restrict__ tally, const double *__restrict__ V,
                           const int *__restrict__ mat, const double *__restrict__ sigt_m,
                           const double *__restrict__ nsf_m, double *__restrict__ phi_internal,
                           double *__restrict__ phi_user, const int *__restrict__ user_of, double *__restrict__ partials,
                           int R, int G, int Gp) {
    __shared__ double sh[16];
    double acc = 0.0;
    const uint32_t n = (uint32_t)R * (uint32_t)G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t r = i / (uint32_t)G, g = i - r * (uint32_t)G;
        const int m = mat[r];
        const double v = V[r];
        const double st = sigt_m[m * G + g];
        const double ph = kFourPi * (double)xsq[((int64_t)r * Gp + g) * 2 + 1] + tally[(int64_t)r * Gp + g] / (st * v);
        if (phi_internal) phi_internal[i] = ph;
        if (phi_user) phi_user[(int64_t)user_of[r] * G + g] = ph;
        acc += v * nsf_m[m * G + g] * ph;
    }
    if (partials) {
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// sum V F of a flux (for the initial normalisation)
__global__ void k_fission_partials(const double *__restrict__ phi, const double *__restrict__ V, const int *__restrict__ mat,
                                   const double *__restrict__ nsf_m, double *__restrict__ partials, int R, int G) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        const int m = mat[r];
        double F = 0.0;
        for (int g = 0; g < G; ++g) F += nsf_m[m * G + g] * phi[(int64_t)r * G + g];
        acc += V[r] * F;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// partials of sum V Sigma_a phi (absorption), Sigma_a = Sigma_t - sum_g' Sigma_s,g->g'
__global__ void k_absorption_partials(const double *__restrict__ phi, const double *__restrict__ V, const int *__restrict__ mat,
                                      const double *__restrict__ sigt_m, const double *__restrict__ sigs_m,
                                      double *__restrict__ partials, int R, int G) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        const int m = mat[r];
        double a = 0.0;
        for (int g = 0; g < G; ++g) {
            double out = 0.0;
            for (int gp = 0; gp < G; ++gp) out += sigs_m[((int64_t)m * G + g) * G + gp];
            a += (sigt_m[m * G + g] - out) * phi[(int64_t)r * G + g];
        }
        acc += V[r] * a;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// k = (sum of partials_f) / (sum of partials_a), single block
__global__ void k_k_estimate(const double *__restrict__ pf, const double *__restrict__ pa, int nblk, double *__restrict__ scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += pf[i];
        b += pa[i];
    }
    const double sa = block_sum(a, sh);
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) scal[kScalK] = (sb > 0 && sa > 0) ? sa / sb : 1.0;
}

// Single block. mode 0: initial normalisation (f = 1/sum); mode 1: eigenvalue update
// k <- k * sum V F_new (the old iterate has sum V F = 1), f = 1/sum; mode 2: fixed source
// (k = 1, f = 1); mode 3: k already set by the coarse-mesh solve, f = 1/sum. Partials are
// summed in a fixed order (deterministic).
__global__ void k_eigen_update(const double *__restrict__ partials, int nblk, double *__restrict__ scal, int mode) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partials[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        scal[kScalFsum] = s;
        if (mode == 0) {
            scal[kScalF] = 1.0 / s;
        } else if (mode == 1) {
            scal[kScalKPrev] = scal[kScalK];
            scal[kScalK] = scal[kScalK] * s;
            scal[kScalF] = 1.0 / s;
        } else if (mode == 2) {
            scal[kScalKPrev] = scal[kScalK];
            scal[kScalF] = 1.0;
        } else {
            scal[kScalF] = 1.0 / s;
        }
    }
}

// phi_new *= f; partials of sum V (phi_new - phi_old)^2 and sum V phi_new^2 (one thread
// per (region, group))
__global__ void k_norm_residual(double *__restrict__ phi_new, const double *__restrict__ phi_old,
                                const double *__restrict__ V, const double *__restrict__ scal,
                                double *__restrict__ partials, int R, int G) {
    __shared__ double sh[16];
    const double f = scal[kScalF];
    double num = 0.0, den = 0.0;
    const uint32_t n = (uint32_t)R * (uint32_t)G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double v = V[i / (uint32_t)G];
        const double x = phi_new[i] * f;
        phi_new[i] = x;
        const double d = x - phi_old[i];
        num += v * d * d;
        den += v * x * x;
    }
    const double a = block_sum(num, sh);
    const double b = block_sum(den, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_residual(const double *__restrict__ partials, int nblk, double *__restrict__ scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    const double sa = block_sum(a, sh);
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        scal[kScalRes] = sb > 0 ? sqrt(sa / sb) : 0.0;
        scal[kScalDk] = fabs(scal[kScalK] - scal[kScalKPrev]);
    }
}

// canonical [T][2][P][G] FP64 <-> internal psi
template <typename Real>
__global__ void k_psi_canon(double *__restrict__ canon, Real *__restrict__ psi, const int *__restrict__ slot_of_canon, int T,
                            int P, int G, int Gp, int nslots, int to_canon) {
    const int64_t n = (int64_t)T * 2 * P * G;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = int(i % G);
        const int p = int((i / G) % P);
        const int s = int((i / ((int64_t)G * P)) % 2);
        const int t = int(i / ((int64_t)G * P * 2));
        const int64_t j = (int64_t)((s * P + p) * Gp + g) * nslots + slot_of_canon[t];
        if (to_canon)
            canon[i] = (double)psi[j];
        else
            psi[j] = (Real)canon[i];
    }
}

// Boundary flux from a scalar-flux guess: psi = phi(r_entry)/(4 pi) for every incoming
// track-sense (r_entry: internal region of the first segment along that sense).
template <typename Real>
__global__ void k_psi_from_phi(const double *__restrict__ phi, const int *__restrict__ entry_region, Real *__restrict__ psi,
                               int P, int G, int Gp, int nslots) {
    const int64_t n = (int64_t)2 * P * Gp * nslots;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int slot = int(i % nslots);
        const int g = int((i / nslots) % Gp);
        const int s = int(i / ((int64_t)nslots * Gp * P));
        const int r = entry_region[s * nslots + slot];
        psi[i] = (r >= 0 && g < G) ? (Real)(phi[(int64_t)r * G + g] / kFourPi) : Real(0);
    }
}

// user <-> internal region order for [R][G] FP64 arrays
__global__ void k_permute_rows(const double *__restrict__ src, double *__restrict__ dst, const int *__restrict__ user_of, int R,
                               int G, int to_user) {
    const int64_t n = (int64_t)R * G;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = int(i / G), g = int(i - (int64_t)r * G);
        const int64_t u = (int64_t)user_of[r] * G + g;
        if (to_user)
            dst[u] = src[i];
        else
            dst[i] = src[u];
    }
}

// validity of a guess: counts of non-finite or negative entries and the number of
// positive entries
__global__ void k_check_guess(const double *__restrict__ x, int64_t n, double *__restrict__ out) {
    __shared__ double sh[16];
    double bad = 0.0, pos = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i];
        if (!isfinite(v) || v < 0) bad += 1.0;
        if (v > 0) pos += 1.0;
    }
    const double a = block_sum(bad, sh);
    const double b = block_sum(pos, sh);
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], a);
        atomicAdd(&out[1], b);
    }
}

// Per-group bound of the FP32 sweep's fluxes: tally_bound[g] = max over regions of |qhat|
// and over the incoming boundary fluxes of |psi| (float bit patterns of non-negative
// values order like the values). Maxima are kept in registers and meet in LDS only at the
// end (a per-element LDS maximum on the block's Gp words serialised: 126 us per sweep at
// 30 M elements): for qhat each thread keeps one group (thread t takes group t mod Gp of
// every (T / Gp)-th region, T the grid's threads); psi is stored as 2 P Gp rows of nslots
// slots, one group per row, and the whole grid walks the rows in order, so each row's
// maximum is folded into LDS once per wave. No 64-bit index division anywhere. The
// caller zeroes tally_bound.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, 64));
    return v;
}

__global__ __launch_bounds__(1024) void k_tally_bound(const float *__restrict__ xsq, const float *__restrict__ psi, int R,
                                                      int Gp, int nrows, int nslots, unsigned *__restrict__ bound) {
    extern __shared__ unsigned bmax[];
    for (int g = threadIdx.x; g < Gp; g += blockDim.x) bmax[g] = 0u;
    __syncthreads();
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t Tg = T / Gp;
    if (tid < Tg * Gp) {
        const int g = int(tid % Gp);
        unsigned m = 0u;
#pragma unroll 4
        for (int64_t r = tid / Gp; r < R; r += Tg) m = max(m, __float_as_uint(fabsf(xsq[2 * (r * Gp + g) + 1])));
        if (m) atomicMax(&bmax[g], m);
    }
    for (int q = 0; q < nrows; ++q) {
        const float *row = psi + (int64_t)q * nslots;
        unsigned m = 0u;
#pragma unroll 4
        for (int64_t j = tid; j < nslots; j += T) m = max(m, __float_as_uint(fabsf(row[j])));
        const unsigned w = wave_max_u32(m);
        if ((threadIdx.x & 63) == 0 && w) atomicMax(&bmax[q % Gp], w);
    }
    __syncthreads();
    for (int g = threadIdx.x; g < Gp; g += blockDim.x)
        if (bmax[g]) atomicMax(&bound[g], bmax[g]);
}

template <typename T> __global__ void k_fill_u32(T *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = T(0);
}

// ---------------------------------------------------------------- launchers
static inline int grid_for(int64_t n, int block, int cap = 4096) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#define MOC_CHECK_LAUNCH()                                                      \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) throw Error(MOC_EHIP, hipGetErrorString(e_));     \
    } while (0)

template <typename Real, int NP, int GB, int MODE, bool CUR>
static void sweep_inst(const SweepArgs &a, int nb, int n_gb, hipStream_t s) {
    if (a.cap > kMaxSlots) throw Error(MOC_EINVAL, "sweep: window slot count above the kernel maximum");
    static_assert(GB <= SweepLds<Real, GB, MODE>::kScaleSlots, "group batch above the scale slots");
    const size_t lds = SweepLds<Real, GB, MODE>::bytes(a.cap);
    if (lds > 64 * 1024) throw Error(MOC_EINVAL, "sweep: tally window does not fit in LDS");
    hipLaunchKernelGGL((k_sweep<Real, NP, GB, MODE, CUR>), dim3(nb, 2, n_gb), dim3(64), lds, s, a);
}

template <typename Real, int NP, int MODE, bool CUR>
static bool sweep_gb(const SweepArgs &a, int nb, int gb, int n_gb, hipStream_t s) {
    switch (gb) {
        case 1: sweep_inst<Real, NP, 1, MODE, CUR>(a, nb, n_gb, s); return true;
        case 2: sweep_inst<Real, NP, 2, MODE, CUR>(a, nb, n_gb, s); return true;
        case 4: sweep_inst<Real, NP, 4, MODE, CUR>(a, nb, n_gb, s); return true;
        case 7: sweep_inst<Real, NP, 7, MODE, CUR>(a, nb, n_gb, s); return true;
        case 8: sweep_inst<Real, NP, 8, MODE, CUR>(a, nb, n_gb, s); return true;
        case 11: sweep_inst<Real, NP, 11, MODE, CUR>(a, nb, n_gb, s); return true;
        default: return false;
    }
}

template <typename Real, int MODE, bool CUR>
static bool sweep_np(const SweepArgs &a, int nb, int np, int gb, int n_gb, hipStream_t s) {
    switch (np) {
        case 1: return sweep_gb<Real, 1, MODE, CUR>(a, nb, gb, n_gb, s);
        case 2: return sweep_gb<Real, 2, MODE, CUR>(a, nb, gb, n_gb, s);
        case 3: return sweep_gb<Real, 3, MODE, CUR>(a, nb, gb, n_gb, s);
        case 4: return sweep_gb<Real, 4, MODE, CUR>(a, nb, gb, n_gb, s);
        default: return false;
    }
}

void launch_sweep(const SweepArgs &a, int precision, int exp_mode, bool currents, int nb, int np, int gb, int n_gb,
                  hipStream_t s) {
    bool ok;
    if (currents) {
        // coarse-surface currents: FP64, or FP32 with the default exponential
        if (precision == MOC_PREC_F64)
            ok = sweep_np<double, MOC_EXP_POLY, true>(a, nb, np, gb, n_gb, s);
        else if (exp_mode == MOC_EXP_POLY)
            ok = sweep_np<float, MOC_EXP_POLY, true>(a, nb, np, gb, n_gb, s);
        else if (exp_mode == MOC_EXP_DIFF)
            ok = sweep_np<float, MOC_EXP_DIFF, true>(a, nb, np, gb, n_gb, s);
        else
            throw Error(MOC_EINVAL, "sweep: coarse-surface currents need MOC_EXP_POLY or MOC_EXP_DIFF");
    } else if (precision == MOC_PREC_F64) {
        ok = sweep_np<double, MOC_EXP_POLY, false>(a, nb, np, gb, n_gb, s);
    } else if (exp_mode == MOC_EXP_TABLE) {
        ok = sweep_np<float, MOC_EXP_TABLE, false>(a, nb, np, gb, n_gb, s);
    } else if (exp_mode == MOC_EXP_LIBM) {
        ok = sweep_np<float, MOC_EXP_LIBM, false>(a, nb, np, gb, n_gb, s);
    } else if (exp_mode == MOC_EXP_DIFF) {
        ok = sweep_np<float, MOC_EXP_DIFF, false>(a, nb, np, gb, n_gb, s);
    } else {
        ok = sweep_np<float, MOC_EXP_POLY, false>(a, nb, np, gb, n_gb, s);
    }
    if (!ok) throw Error(MOC_EINVAL, "sweep: no kernel instance for this polar count / group batch");
    MOC_CHECK_LAUNCH();
}

void launch_tally_bound(const DevProblem &d, const void *psi_in, hipStream_t s) {
    if (d.precision != MOC_PREC_F32) return;
    const int64_t npsi = (int64_t)2 * d.P * d.Gp * d.nslots;
    hipLaunchKernelGGL(k_fill_u32<unsigned>, dim3(1), dim3(64), 0, s, d.tally_bound, (int64_t)d.Gp);
    const size_t lds = sizeof(unsigned) * (size_t)d.Gp;
    if (lds > 64 * 1024) throw Error(MOC_EINVAL, "sweep: too many groups for the flux bound");
    // few blocks: every block ends with one global atomic per group on the same Gp words
    const int nblk = grid_for((int64_t)d.R * d.Gp + npsi, 1024, 256);
    hipLaunchKernelGGL(k_tally_bound, dim3(nblk), dim3(1024), lds, s, (const float *)d.xsq, (const float *)psi_in, d.R,
                       d.Gp, 2 * d.P * d.Gp, d.nslots, d.tally_bound);
    MOC_CHECK_LAUNCH();
}

void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    MOC_CHECK_LAUNCH();
}

void launch_fill_real(void *p, int64_t n, int precision, hipStream_t s) {
    if (precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, (double *)p, n, 0.0);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, (float *)p, n, 0.0f);
    MOC_CHECK_LAUNCH();
}

void launch_scale_real(void *p, int64_t n, int precision, const double *f, hipStream_t s) {
    if (precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_scale<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, (double *)p, n, f);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, (float *)p, n, f);
    MOC_CHECK_LAUNCH();
}

void launch_scale_f64(double *p, int64_t n, const double *f, hipStream_t s) {
    hipLaunchKernelGGL(k_scale<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, f);
    MOC_CHECK_LAUNCH();
}

void launch_prep_user(const DevProblem &d, const double *src_user, hipStream_t s) {
    const int64_t n = (int64_t)d.R * d.Gp;
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_prep_user<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, src_user, d.user_of, d.mat, d.sigt_m,
                           (double *)d.xsq, d.R, d.G, d.Gp);
    else
        hipLaunchKernelGGL(k_prep_user<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, src_user, d.user_of, d.mat, d.sigt_m,
                           (float *)d.xsq, d.R, d.G, d.Gp);
    MOC_CHECK_LAUNCH();
}

void launch_source(const DevProblem &d, const double *phi, hipStream_t s) {
    const int grid = grid_for((int64_t)d.R * d.G, 256, 8192);
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_source<double>, dim3(grid), dim3(256), 0, s, phi, d.scal, d.mat, d.sigt_m, d.sigs_m, d.nsf_m,
                           d.chi_m, d.qext, (double *)d.xsq, d.R, d.G, d.Gp);
    else
        hipLaunchKernelGGL(k_source<float>, dim3(grid), dim3(256), 0, s, phi, d.scal, d.mat, d.sigt_m, d.sigs_m, d.nsf_m,
                           d.chi_m, d.qext, (float *)d.xsq, d.R, d.G, d.Gp);
    MOC_CHECK_LAUNCH();
}

void launch_finalize(const DevProblem &d, double *phi_internal, double *phi_user, double *partials, hipStream_t s) {
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_finalize<double>, dim3(kReduceBlocks), dim3(256), 0, s, (const double *)d.xsq, d.tally, d.V, d.mat,
                           d.sigt_m, d.nsf_m, phi_internal, phi_user, d.user_of, partials, d.R, d.G, d.Gp);
    else
        hipLaunchKernelGGL(k_finalize<float>, dim3(kReduceBlocks), dim3(256), 0, s, (const float *)d.xsq, d.tally, d.V, d.mat,
                           d.sigt_m, d.nsf_m, phi_internal, phi_user, d.user_of, partials, d.R, d.G, d.Gp);
    MOC_CHECK_LAUNCH();
}

void launch_fission_partials(const DevProblem &d, const double *phi, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_fission_partials, dim3(kReduceBlocks), dim3(256), 0, s, phi, d.V, d.mat, d.nsf_m, partials, d.R, d.G);
    MOC_CHECK_LAUNCH();
}

void launch_k_estimate(const DevProblem &d, const double *phi, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_fission_partials, dim3(kReduceBlocks), dim3(256), 0, s, phi, d.V, d.mat, d.nsf_m, partials, d.R, d.G);
    hipLaunchKernelGGL(k_absorption_partials, dim3(kReduceBlocks), dim3(256), 0, s, phi, d.V, d.mat, d.sigt_m, d.sigs_m,
                       partials + kReduceBlocks, d.R, d.G);
    hipLaunchKernelGGL(k_k_estimate, dim3(1), dim3(256), 0, s, partials, partials + kReduceBlocks, kReduceBlocks, d.scal);
    MOC_CHECK_LAUNCH();
}

void launch_eigen_update(const DevProblem &d, const double *partials, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_eigen_update, dim3(1), dim3(256), 0, s, partials, kReduceBlocks, d.scal, mode);
    MOC_CHECK_LAUNCH();
}

void launch_norm_residual(const DevProblem &d, double *phi_new, const double *phi_old, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_residual, dim3(kReduceBlocks), dim3(256), 0, s, phi_new, phi_old, d.V, d.scal, partials, d.R, d.G);
    hipLaunchKernelGGL(k_residual, dim3(1), dim3(256), 0, s, partials, kReduceBlocks, d.scal);
    MOC_CHECK_LAUNCH();
}

void launch_psi_canon(const DevProblem &d, double *canon, void *psi, int to_canon, hipStream_t s) {
    const int64_t n = (int64_t)d.T * 2 * d.P * d.G;
    if (n == 0) return;
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_psi_canon<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, canon, (double *)psi, d.slot_of_canon,
                           d.T, d.P, d.G, d.Gp, d.nslots, to_canon);
    else
        hipLaunchKernelGGL(k_psi_canon<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, canon, (float *)psi, d.slot_of_canon,
                           d.T, d.P, d.G, d.Gp, d.nslots, to_canon);
    MOC_CHECK_LAUNCH();
}

void launch_psi_from_phi(const DevProblem &d, const double *phi_internal, void *psi, hipStream_t s) {
    const int64_t n = (int64_t)2 * d.P * d.Gp * d.nslots;
    if (d.precision == MOC_PREC_F64)
        hipLaunchKernelGGL(k_psi_from_phi<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, phi_internal, d.entry_region,
                           (double *)psi, d.P, d.G, d.Gp, d.nslots);
    else
        hipLaunchKernelGGL(k_psi_from_phi<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, phi_internal, d.entry_region,
                           (float *)psi, d.P, d.G, d.Gp, d.nslots);
    MOC_CHECK_LAUNCH();
}

void launch_permute_rows(const DevProblem &d, const double *src, double *dst, int to_user, hipStream_t s) {
    const int64_t n = (int64_t)d.R * d.G;
    hipLaunchKernelGGL(k_permute_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, d.user_of, d.R, d.G, to_user);
    MOC_CHECK_LAUNCH();
}

void launch_check_guess(const double *x, int64_t n, double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, s, out2, (int64_t)2, 0.0);
    hipLaunchKernelGGL(k_check_guess, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, out2);
    MOC_CHECK_LAUNCH();
}

}  // namespace moc
