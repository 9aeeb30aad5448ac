// HIP kernels of libmoc's DGMOC solver for gfx950 (CDNA4): driven flux, plane sweep with
// the 2x2 exponential segment solution, face-flux store, source, finalisation and the
// FP64 reductions of the power iteration.
//
// Discretisation (Sec. 2.1.1, Eqs. DGMOC_expansion / DGMOC_weak_up, linear order): in a
// plane of height h, along a 2D segment of length l, direction with polar cosine mu and
// sine sin(theta), the Legendre coefficients Psi = (psi_0, psi_1) obey, in the ward's
// local orientation (the downward ward mirrors xi),
//     sin(theta) dPsi/ds = -A Psi + Q,   A = Sigma_t I + kappa K,   kappa = mu / h,
//     K = [[1, 1], [-3, 3]],             Q = (q_0 + kappa psi_f, q_1 - 3 kappa psi_f),
// psi_f the flux entering through the upwind face. With the driven flux
// D = A^-1 Q (constant along the segment) and X = Psi_in - D, the exact solution is
//     Psi_out = Psi_in - (I - e^-M) X,   Psi_bar = D + M^-1 (I - e^-M) X,   M = (l / sin) A.
// K = 2 I + J with J = [[-1, 1], [-3, 1]], J^2 = -2 I, so M = a I + b J with
// a = tau + 2 beta, b = beta (tau = Sigma_t l / sin, beta = kappa l / sin), and any
// function of M is Re f(z) I + Im f(z) / sqrt(2) J at z = a + i c, c = sqrt(2) beta.
// Hence, with e = e^-a, N1 = 1 - e cos c = (1 - e) + e (1 - cos c), N2 = e sin c:
//     I - e^-M = N1 I + N2 / sqrt(2) J
//     M^-1 (I - e^-M) = [(a N1 + c N2) I + (a N2 - c N1) / sqrt(2) J] / (a^2 + c^2)
// 1 - e and 1 - cos c = 2 sin^2(c / 2) are formed with relative accuracy, so short
// segments keep full relative accuracy (as the planar sweep's 1 - e^-tau does).
//
// Layouts (internal region order r):
//   sigt3 : Real [Nz][R][Gp]            q3   : Real [Nz][R][Gp][2] (per steradian)
//   drv   : Real [2 NAb][R][n_gb][P][gb][2], direction index (a - a0) * 2 + sense
//   face  : Real [2 NAb][P][R][Gp]      raw tallies sum delta_a l (psi_bar_0 + psi_bar_1)
//   bot   : Real [2 NA][P][R][Gp]       face flux through the bottom (reflective bottom)
//   tally : double [Nz][R][Gp][2]       phi : double [Nz][R][G][2]
//   psi   : Real [2 wards][Nz][2 senses][P][2][Gp][nslots]
#include <cmath>

#include "dg_kernels.h"
#include "moc_expf.h"
#include "moc_pack.h"

namespace moc {

static constexpr double kFourPiDg = 12.566370614359172953850573533118;
static constexpr double kInvSqrt2 = 0.70710678118654752440;

template <typename Real> struct DgSeg;
template <> struct DgSeg<float> { using type = SegF; };
template <> struct DgSeg<double> { using type = SegD; };

// sin and cos of x >= 0 with relative accuracy for small x: x = n pi/2 + r, |r| <= pi/4
// by a two-constant Cody-Waite reduction, Taylor polynomials in r (truncation below
// 2e-9 relative), quadrant from n.
__device__ __forceinline__ void dg_sincos(float x, float &sn, float &cs) {
    const float n = rintf(x * 0.63661977236758134f);
    float r = fmaf(-n, 1.5707963705062866f, x);
    r = fmaf(-n, -4.3711390001862427e-8f, r);
    const float r2 = r * r;
    const float s = r * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
    const float c =
        1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
    const int q = (int)n;
    const float ss = (q & 1) ? c : s, cc = (q & 1) ? s : c;
    sn = (q & 2) ? -ss : ss;
    cs = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void dg_sincos(double x, double &sn, double &cs) { sincos(x, &sn, &cs); }

// The same for a whole wavefront: when every lane has x <= pi/4 (the usual case: c / 2
// is below that for segments shorter than about 1.1 h sin(theta) / mu) the reduction is
// the identity and the polynomials alone give the result; otherwise the full reduction.
__device__ __forceinline__ void dg_sincos_wave(float x, float &sn, float &cs) {
    if (__all(x <= 0.78539816f)) {
        const float r2 = x * x;
        sn = x * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
        cs = 1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
    } else {
        dg_sincos(x, sn, cs);
    }
}
__device__ __forceinline__ void dg_sincos_wave(double x, double &sn, double &cs) { sincos(x, &sn, &cs); }

// 1 - e^-a for a >= 0 with relative accuracy
__device__ __forceinline__ float dg_one_minus_exp(float a) { return one_minus_exp2_poly(a * -1.4426950408889634f); }
__device__ __forceinline__ double dg_one_minus_exp(double a) { return -expm1(-a); }

__device__ __forceinline__ float dg_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double dg_rcp(double x) { return 1.0 / x; }

// ---------------------------------------------------------------- driven flux
// Alg. DGMOC_sweep's driven-flux step: for every direction of the block, region and
// group, the face flux entering the plane (none, the previous plane's face tally over the
// per-angle track area, or the bottom buffer) and D = A^-1 Q. The face tallies are
// cleared for the plane's own sweep.
template <typename Real> __global__ void k_dg_driven(DgDrivenArgs a) {
    // grid: x over the (region, group) entries of one row, y = direction * P + polar
    const int rowlen = a.R * a.Gp;
    const int p = blockIdx.y % a.P, dirb = blockIdx.y / a.P;
    const int ang = a.a0 + (dirb >> 1);
    const Real *__restrict__ sigt = reinterpret_cast<const Real *>(a.sigt);
    const Real *__restrict__ q = reinterpret_cast<const Real *>(a.q);
    Real *__restrict__ face = reinterpret_cast<Real *>(a.face);
    const Real *__restrict__ bot = reinterpret_cast<const Real *>(a.bot);
    const Real *__restrict__ inv_va = reinterpret_cast<const Real *>(a.inv_va);
    Real *__restrict__ drv = reinterpret_cast<Real *>(a.drv);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rowlen; e += gridDim.x * blockDim.x) {
        const int r = e / a.Gp, g = e - r * a.Gp;
        const int64_t i = (int64_t)blockIdx.y * rowlen + e;
        // arithmetic in the sweep precision (the result is stored in it); every term of
        // det is positive
        Real pf = 0;
        if (a.mode == 1)
            pf = face[i] * inv_va[(int64_t)ang * a.R + r];
        else if (a.mode == 2)
            pf = bot[(((int64_t)(a.a0 * 2 + dirb) * a.P + p) * a.R + r) * a.Gp + g];
        face[i] = Real(0);
        const Real st = sigt[(int64_t)r * a.Gp + g];
        const Real k = (Real)a.kap[p];
        const Real q0 = q[((int64_t)r * a.Gp + g) * 2] + k * pf;
        const Real q1 = (Real)a.sgn * q[((int64_t)r * a.Gp + g) * 2 + 1] - Real(3) * k * pf;
        const Real rdet = dg_rcp(st * st + Real(4) * st * k + Real(6) * k * k);
        const Real d0 = ((st + Real(3) * k) * q0 - k * q1) * rdet;
        const Real d1 = (Real(3) * k * q0 + (st + k) * q1) * rdet;
        const int gbi = g / a.gb, j = g - gbi * a.gb;
        const int64_t o = ((((int64_t)dirb * a.R + r) * a.n_gb + gbi) * a.P + p) * a.gb + j;
        if (gbi < a.n_gb) {
            drv[2 * o] = d0;
            drv[2 * o + 1] = d1;
        }
    }
}

// After the downward ward's last (bottom) plane: the face tallies over the per-angle
// track area are the flux leaving through the bottom, kept for the next sweep's upward
// ward (reflective bottom).
template <typename Real> __global__ void k_dg_store_bottom(DgDrivenArgs a) {
    const int rowlen = a.R * a.Gp;
    const int dirb = blockIdx.y / a.P;
    const int ang = a.a0 + (dirb >> 1);
    const Real *__restrict__ face = reinterpret_cast<const Real *>(a.face);
    Real *__restrict__ bot = const_cast<Real *>(reinterpret_cast<const Real *>(a.bot));
    const Real *__restrict__ inv_va = reinterpret_cast<const Real *>(a.inv_va);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rowlen; e += gridDim.x * blockDim.x) {
        const int r = e / a.Gp;
        const int64_t i = (int64_t)blockIdx.y * rowlen + e;
        bot[(int64_t)a.a0 * 2 * a.P * rowlen + i] = face[i] * inv_va[(int64_t)ang * a.R + r];
    }
}

// ---------------------------------------------------------------- plane sweep
// One wavefront = one batch of 64 adjacent parallel tracks of one angle, one sense and
// one group batch [g0, g0 + GB), in one plane and ward. Lane l walks track l through the
// batch's tally windows as in the planar sweep; per segment, polar angle and group it
// applies the exact 2x2 segment solution (header comment). Segment averages go, weighted,
// into a window-local FP64 LDS tally per slot and group: both scalar-flux moments
// (polar-summed in registers) and, per polar angle, the face tally of the direction;
// each window's slots are flushed with one global atomic per value.
template <typename Real, int NP, int GB> __global__ __launch_bounds__(64) void k_dg_sweep(DgSweepArgs args) {
    using Seg = typename DgSeg<Real>::type;
    constexpr int NV = 2 + NP;   // LDS values per (slot, group): moments 0, 1, face per polar
    extern __shared__ unsigned char smem[];
    double *tl = reinterpret_cast<double *>(smem);   // [cap][GB][NV]
    const int cap = args.cap;
    int *tabl = reinterpret_cast<int *>(smem + sizeof(double) * GB * NV * cap);
    for (int i = threadIdx.x; i < GB * NV * cap; i += 64) tl[i] = 0.0;
    __syncthreads();

    const int b = args.b0 + blockIdx.x, sense = blockIdx.y, gbi = blockIdx.z, lane = threadIdx.x;
    const int nslots = args.nslots, Gp = args.Gp, R = args.R, n_gb = args.n_gb;
    const int slot = b * 64 + lane;
    const int g0 = gbi * GB;
    const int ang = args.batch_angle[b];
    const int dirb = (ang - args.a0) * 2 + sense;
    const Seg *__restrict__ segs = reinterpret_cast<const Seg *>(args.segs);
    const Real *__restrict__ psi_in = reinterpret_cast<const Real *>(args.psi_in);
    Real *__restrict__ psi_out = reinterpret_cast<Real *>(args.psi_out);
    const Real *__restrict__ sigt = reinterpret_cast<const Real *>(args.sigt);
    const Real *__restrict__ drv = reinterpret_cast<const Real *>(args.drv);
    double *__restrict__ tally = args.tally;
    Real *__restrict__ face = reinterpret_cast<Real *>(args.face);

    // per polar angle: 1/sin, kappa, moment weights (moment 1 mirrored in the downward ward)
    const Real *__restrict__ wdir = reinterpret_cast<const Real *>(args.wdir);
    const Real *__restrict__ inv_sin = reinterpret_cast<const Real *>(args.inv_sin);
    Real is[NP], kp[NP], cw0[NP], cw1[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        is[p] = inv_sin[p];
        kp[p] = (Real)args.kap[p];
        cw0[p] = wdir[ang * NP + p];
        cw1[p] = cw0[p] * (Real)args.sgn;
    }
    const Real dl = reinterpret_cast<const Real *>(args.dlt)[ang];

    Real ps[NP][GB][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < GB; ++j)
#pragma unroll
            for (int m = 0; m < 2; ++m)
                ps[p][j][m] = psi_in[(int64_t)(((sense * NP + p) * 2 + m) * Gp + g0 + j) * nslots + slot];

    struct Data {
        Real st[GB];
        Real d[NP][GB][2];
    };
    // per-wave bases; a region's rows are then 32-bit offsets from them
    const Real *__restrict__ sigt_w = sigt + g0;
    const Real *__restrict__ drv_w = drv + ((int64_t)dirb * R * n_gb + gbi) * (NP * GB * 2);
    const uint32_t drv_rs = (uint32_t)n_gb * (NP * GB * 2);
    auto load = [&](uint32_t key, Data &x) {
        const uint32_t r = key >> kSlotBits;
        const Real *srow = sigt_w + r * (uint32_t)Gp;
        const Real *drow = drv_w + r * drv_rs;
        if constexpr (sizeof(Real) == 4 && GB == 4) {
            const float4 v = *reinterpret_cast<const float4 *>(srow);
            x.st[0] = v.x; x.st[1] = v.y; x.st[2] = v.z; x.st[3] = v.w;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float4 u = reinterpret_cast<const float4 *>(drow)[2 * p];
                const float4 w = reinterpret_cast<const float4 *>(drow)[2 * p + 1];
                x.d[p][0][0] = u.x; x.d[p][0][1] = u.y; x.d[p][1][0] = u.z; x.d[p][1][1] = u.w;
                x.d[p][2][0] = w.x; x.d[p][2][1] = w.y; x.d[p][3][0] = w.z; x.d[p][3][1] = w.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < GB; ++j) x.st[j] = srow[j];
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int j = 0; j < GB; ++j) {
                    x.d[p][j][0] = drow[(p * GB + j) * 2];
                    x.d[p][j][1] = drow[(p * GB + j) * 2 + 1];
                }
        }
    };

    const int64_t w0 = args.batch_win[b], w1 = args.batch_win[b + 1];
    for (int64_t wi = 0; wi < w1 - w0; ++wi) {
        const int64_t w = sense ? w1 - 1 - wi : w0 + wi;
        const int n = args.win_nsteps[w];
        const Seg *__restrict__ ws = segs + args.win_entry_off[w];
        const int ns = args.win_nslots[w];
        const int *__restrict__ tab = args.win_tab + args.win_tab_off[w];
        int tabv[kMaxSlots / 64];
#pragma unroll
        for (int u = 0; u < kMaxSlots / 64; ++u) tabv[u] = (u * 64 + lane < ns) ? tab[u * 64 + lane] : 0;
        auto step_of = [&](int i) { return (int64_t)(sense ? n - 1 - i : i) * 64 + lane; };
        auto clampi = [&](int i) { return i < n ? i : n - 1; };

        // one step. Psi_in - Psi_out = (I - e^-M) X = N1 X + N2 / sqrt(2) J X, and the segment
        // average is D + M^-1 (Psi_in - Psi_out) with M^-1 = (a I - b J) / (a^2 + c^2).
        // Padding steps (length 0) leave psi unchanged and add exact zeros; their lanes add
        // them to the window's slots spread by lane (one shared row would serialise them),
        // which keeps the tally atomics free of per-lane branches.
        double *pad_row = tl + (lane % (ns > 0 ? ns : 1)) * (GB * NV);
        auto update = [&](const Seg &sg, const Data &x) {
            const Real len = sg.len;
            const int ts = int(sg.key & ((1u << kSlotBits) - 1));
            double *row = len > Real(0) ? tl + ts * (GB * NV) : pad_row;
            Real acc0[GB], acc1[GB];
#pragma unroll
            for (int j = 0; j < GB; ++j) acc0[j] = acc1[j] = Real(0);
            const Real dll = dl * len;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const Real lp = len * is[p];
                const Real bt = kp[p] * lp;
                const Real c = Real(1.4142135623730951) * bt;
                Real sh, ch;
                dg_sincos_wave(Real(kInvSqrt2) * bt, sh, ch);   // sin and cos of c / 2
                const Real scs = Real(1.4142135623730951) * sh * ch;   // sin(c) / sqrt(2)
                const Real omc = Real(2) * sh * sh;                     // 1 - cos(c)
                const Real c2 = c * c, b2 = bt + bt;
                const Real w0p = cw0[p] * len, w1p = cw1[p] * len;
#pragma unroll
                for (int j = 0; j < GB; ++j) {
                    const Real aa = x.st[j] * lp + b2;
                    const Real F = dg_one_minus_exp(aa);
                    const Real e = Real(1) - F;
                    const Real N1 = e * omc + F, N2s = e * scs;
                    const Real X0 = ps[p][j][0] - x.d[p][j][0], X1 = ps[p][j][1] - x.d[p][j][1];
                    const Real D0 = N1 * X0 + N2s * (X1 - X0);
                    const Real D1 = N1 * X1 + N2s * (X1 - Real(3) * X0);
                    ps[p][j][0] -= D0;
                    ps[p][j][1] -= D1;
                    Real den = aa * aa + c2;
                    den = den > Real(1e-30) ? den : Real(1e-30);
                    const Real rd = dg_rcp(den);
                    const Real b0 = x.d[p][j][0] + rd * (aa * D0 - bt * (D1 - D0));
                    const Real b1 = x.d[p][j][1] + rd * (aa * D1 - bt * (D1 - Real(3) * D0));
                    acc0[j] += w0p * b0;
                    acc1[j] += w1p * b1;
                    atomicAdd(&row[j * NV + 2 + p], (double)(dll * (b0 + b1)));
                }
            }
#pragma unroll
            for (int j = 0; j < GB; ++j) {
                atomicAdd(&row[j * NV], (double)acc0[j]);
                atomicAdd(&row[j * NV + 1], (double)acc1[j]);
            }
        };
        // software pipeline, unrolled by two so that the two data sets alternate without
        // copies: segment entries two steps ahead, cross sections and driven flux one
        Seg s0 = ws[step_of(0)], s1 = ws[step_of(clampi(1))];
        Data x0, x1;
        load(s0.key, x0);
        for (int i = 0; i < n; i += 2) {
            const Seg s2 = ws[step_of(clampi(i + 2))];
            load(s1.key, x1);
            update(s0, x0);
            if (i + 1 < n) {
                const Seg s3 = ws[step_of(clampi(i + 3))];
                load(s2.key, x0);
                update(s1, x1);
                s0 = s2;
                s1 = s3;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxSlots / 64; ++u)
            if (u * 64 + lane < ns) tabl[u * 64 + lane] = tabv[u];
        __syncthreads();
        // flush: (slot, group, value) triples, values fastest
        for (int e = lane; e < ns * GB * NV; e += 64) {
            const double v = tl[e];
            if (v != 0.0) {
                const int sl = e / (GB * NV), rem = e - sl * (GB * NV);
                const int j = rem / NV, cidx = rem - j * NV;
                const int reg = tabl[sl];
                if (cidx < 2)
                    unsafeAtomicAdd(&tally[((int64_t)reg * Gp + g0 + j) * 2 + cidx], v);
                else
                    unsafeAtomicAdd(&face[(((int64_t)dirb * NP + (cidx - 2)) * R + reg) * Gp + g0 + j], (Real)v);
                tl[e] = 0.0;
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
            for (int j = 0; j < GB; ++j)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    psi_out[(int64_t)(((s2 * NP + p) * 2 + m) * Gp + g0 + j) * nslots + slot2] = ps[p][j][m];
    }
    if (!args.fed[sense * nslots + slot]) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int j = 0; j < GB; ++j)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    psi_out[(int64_t)(((sense * NP + p) * 2 + m) * Gp + g0 + j) * nslots + slot] = Real(0);
    }
}

// ---------------------------------------------------------------- source, finalise
__device__ __forceinline__ double dg_block_sum(double v, double *sh) {
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

// q = s / (4 pi) per moment from a caller's emission density (user order)
template <typename Real>
__global__ void k_dg_prep_user(const double *__restrict__ src, const int *__restrict__ user_of, Real *__restrict__ q3, int Nz,
                               int R, int G, int Gp) {
    const int64_t n = (int64_t)Nz * R * Gp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = int(i % Gp);
        const int r = int((i / Gp) % R);
        const int z = int(i / ((int64_t)Gp * R));
        Real v0 = 0, v1 = 0;
        if (g < G) {
            const int64_t u = (((int64_t)z * R + user_of[r]) * G + g) * 2;
            v0 = (Real)(src[u] / kFourPiDg);
            v1 = (Real)(src[u + 1] / kFourPiDg);
        }
        q3[2 * i] = v0;
        q3[2 * i + 1] = v1;
    }
}

// Emission moments (Eq. MGNTE, isotropic scattering; linear in the flux, so each
// moment of the emission is built from the same moment of the flux):
//   s_m = sum_g' Sigma_s,g'->g phi_m,g' + chi_g F_m / k (+ external), F_m = sum nuSigma_f phi_m
// then q = s / (4 pi). FP64 arithmetic.
template <typename Real>
__global__ void k_dg_source(const double *__restrict__ phi, const double *__restrict__ scal, const int *__restrict__ mat3,
                            const double *__restrict__ sigs_m, const double *__restrict__ nsf_m,
                            const double *__restrict__ chi_m, const double *__restrict__ qext, Real *__restrict__ q3,
                            int64_t ncell, int G, int Gp) {
    const double inv_k = 1.0 / scal[kScalK];
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const int m = mat3[c];
        const double *ph = phi + c * G * 2;
        double F0 = 0.0, F1 = 0.0;
        for (int gp = 0; gp < G; ++gp) {
            F0 += nsf_m[m * G + gp] * ph[2 * gp];
            F1 += nsf_m[m * G + gp] * ph[2 * gp + 1];
        }
        for (int g = 0; g < G; ++g) {
            double s0 = chi_m[m * G + g] * F0 * inv_k, s1 = chi_m[m * G + g] * F1 * inv_k;
            const double *col = sigs_m + (int64_t)m * G * G + g;
            for (int gp = 0; gp < G; ++gp) {
                s0 += col[(int64_t)gp * G] * ph[2 * gp];
                s1 += col[(int64_t)gp * G] * ph[2 * gp + 1];
            }
            if (qext) {
                s0 += qext[(c * G + g) * 2];
                s1 += qext[(c * G + g) * 2 + 1];
            }
            q3[(c * Gp + g) * 2] = (Real)(s0 / kFourPiDg);
            q3[(c * Gp + g) * 2 + 1] = (Real)(s1 / kFourPiDg);
        }
    }
}

// phi_m = tally_m / V_r (segment averages already weighted), to the internal flux with
// per-block partials of sum V h nuSigma_f phi_0, or to a user buffer.
__global__ void k_dg_finalize(const double *__restrict__ tally, const double *__restrict__ V, const double *__restrict__ hV,
                              const int *__restrict__ mat3, const double *__restrict__ nsf_m, const int *__restrict__ user_of,
                              double *__restrict__ phi_internal, double *__restrict__ phi_user, double *__restrict__ partials,
                              int Nz, int R, int G, int Gp) {
    __shared__ double sh[16];
    double acc = 0.0;
    const int64_t ncell = (int64_t)Nz * R;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const int r = int(c % R), z = int(c / R);
        const double inv_v = 1.0 / V[r];
        const int m = mat3[c];
        double F = 0.0;
        for (int g = 0; g < G; ++g) {
            const double f0 = tally[(c * Gp + g) * 2] * inv_v, f1 = tally[(c * Gp + g) * 2 + 1] * inv_v;
            if (phi_internal) {
                phi_internal[(c * G + g) * 2] = f0;
                phi_internal[(c * G + g) * 2 + 1] = f1;
            }
            if (phi_user) {
                const int64_t u = (((int64_t)z * R + user_of[r]) * G + g) * 2;
                phi_user[u] = f0;
                phi_user[u + 1] = f1;
            }
            F += nsf_m[m * G + g] * f0;
        }
        acc += hV[c] * F;
    }
    if (partials) {
        const double t = dg_block_sum(acc, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

__global__ void k_dg_fission_partials(const double *__restrict__ phi, const double *__restrict__ hV, const int *__restrict__ mat3,
                                      const double *__restrict__ nsf_m, double *__restrict__ partials, int64_t ncell, int G) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const int m = mat3[c];
        double F = 0.0;
        for (int g = 0; g < G; ++g) F += nsf_m[m * G + g] * phi[(c * G + g) * 2];
        acc += hV[c] * F;
    }
    const double t = dg_block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// phi_new *= f; partials of the squared L2 norms of the linear field's change and of the
// new field (weights V h for moment 0, V h / 3 for moment 1)
__global__ void k_dg_norm_residual(double *__restrict__ phi_new, const double *__restrict__ phi_old,
                                   const double *__restrict__ hV, const double *__restrict__ scal,
                                   double *__restrict__ partials, int64_t ncell, int G) {
    __shared__ double sh[16];
    const double f = scal[kScalF];
    double num = 0.0, den = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const double v = hV[c];
        for (int i = 0; i < 2 * G; ++i) {
            const int64_t k = c * 2 * G + i;
            const double wt = (i & 1) ? v / 3.0 : v;
            const double x = phi_new[k] * f;
            phi_new[k] = x;
            const double d = x - phi_old[k];
            num += wt * d * d;
            den += wt * x * x;
        }
    }
    const double a = dg_block_sum(num, sh);
    const double b = dg_block_sum(den, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_dg_residual(const double *__restrict__ partials, int nblk, double *__restrict__ scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    const double sa = dg_block_sum(a, sh);
    const double sb = dg_block_sum(b, sh);
    if (threadIdx.x == 0) {
        scal[kScalRes] = sb > 0 ? sqrt(sa / sb) : 0.0;
        scal[kScalDk] = fabs(scal[kScalK] - scal[kScalKPrev]);
    }
}

// cold start: moment 0 = 1, moment 1 = 0
__global__ void k_dg_cold(double *__restrict__ phi, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        phi[i] = (i & 1) ? 0.0 : 1.0;
}

// [Nz][R][G][2] between internal and user region order
__global__ void k_dg_permute(const double *__restrict__ src, double *__restrict__ dst, const int *__restrict__ user_of,
                             int Nz, int R, int G, int to_user) {
    const int64_t n = (int64_t)Nz * R * G * 2;
    const int row = 2 * G;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = int(i % row);
        const int r = int((i / row) % R);
        const int z = int(i / ((int64_t)row * R));
        const int64_t u = ((int64_t)z * R + user_of[r]) * row + k;
        if (to_user)
            dst[u] = src[i];
        else
            dst[i] = src[u];
    }
}

// ---------------------------------------------------------------- launchers
static void dg_check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(MOC_EHIP, hipGetErrorString(e));
}

static int grid_for(int64_t n, int block = 256) {
    const int64_t b = (n + block - 1) / block;
    return (int)(b < 1 ? 1 : (b > 65535 * 4 ? 65535 * 4 : b));
}

static dim3 row_grid(const DgDrivenArgs &a) {
    const int64_t rowlen = (int64_t)a.R * a.Gp;
    const int64_t bx = (rowlen + 255) / 256;
    return dim3((unsigned)(bx < 1 ? 1 : (bx > 4096 ? 4096 : bx)), (unsigned)(2 * a.nab * a.P));
}

void launch_dg_driven(const DgDrivenArgs &a, int precision, hipStream_t s) {
    if (precision == MOC_PREC_F64)
        k_dg_driven<double><<<row_grid(a), 256, 0, s>>>(a);
    else
        k_dg_driven<float><<<row_grid(a), 256, 0, s>>>(a);
    dg_check_launch();
}

void launch_dg_store_bottom(const DgDrivenArgs &a, int precision, hipStream_t s) {
    if (precision == MOC_PREC_F64)
        k_dg_store_bottom<double><<<row_grid(a), 256, 0, s>>>(a);
    else
        k_dg_store_bottom<float><<<row_grid(a), 256, 0, s>>>(a);
    dg_check_launch();
}

template <typename Real, int NP, int GB> static void launch_dg_sweep_t(const DgSweepArgs &a, int nb, hipStream_t s) {
    const size_t lds = sizeof(double) * GB * (2 + NP) * (size_t)a.cap + sizeof(int) * (size_t)a.cap;
    hipLaunchKernelGGL((k_dg_sweep<Real, NP, GB>), dim3(nb, 2, a.n_gb), dim3(64), lds, s, a);
}

template <typename Real, int NP> static void launch_dg_sweep_p(const DgSweepArgs &a, int nb, int gb, hipStream_t s) {
    if (gb == 1) launch_dg_sweep_t<Real, NP, 1>(a, nb, s);
    else if (gb == 2) launch_dg_sweep_t<Real, NP, 2>(a, nb, s);
    else launch_dg_sweep_t<Real, NP, 4>(a, nb, s);
}

template <typename Real> static void launch_dg_sweep_r(const DgSweepArgs &a, int nb, int np, int gb, hipStream_t s) {
    switch (np) {
    case 1: launch_dg_sweep_p<Real, 1>(a, nb, gb, s); break;
    case 2: launch_dg_sweep_p<Real, 2>(a, nb, gb, s); break;
    case 3: launch_dg_sweep_p<Real, 3>(a, nb, gb, s); break;
    default: launch_dg_sweep_p<Real, 4>(a, nb, gb, s); break;
    }
}

void launch_dg_sweep(const DgSweepArgs &a, int precision, int nb, int np, int gb, hipStream_t s) {
    if (nb <= 0) return;
    if (precision == MOC_PREC_F64)
        launch_dg_sweep_r<double>(a, nb, np, gb, s);
    else
        launch_dg_sweep_r<float>(a, nb, np, gb, s);
    dg_check_launch();
}

void launch_dg_prep_user(const DevProblem &d, const DevDG &g, const double *src_user, hipStream_t s) {
    const int64_t n = (int64_t)g.Nz * d.R * g.Gp;
    if (d.precision == MOC_PREC_F64)
        k_dg_prep_user<double><<<grid_for(n), 256, 0, s>>>(src_user, d.user_of, (double *)g.q3, g.Nz, d.R, d.G, g.Gp);
    else
        k_dg_prep_user<float><<<grid_for(n), 256, 0, s>>>(src_user, d.user_of, (float *)g.q3, g.Nz, d.R, d.G, g.Gp);
    dg_check_launch();
}

void launch_dg_source(const DevProblem &d, const DevDG &g, const double *phi, hipStream_t s) {
    const int64_t nc = (int64_t)g.Nz * d.R;
    if (d.precision == MOC_PREC_F64)
        k_dg_source<double><<<grid_for(nc), 256, 0, s>>>(phi, d.scal, g.mat3, d.sigs_m, d.nsf_m, d.chi_m, g.qext,
                                                         (double *)g.q3, nc, d.G, g.Gp);
    else
        k_dg_source<float><<<grid_for(nc), 256, 0, s>>>(phi, d.scal, g.mat3, d.sigs_m, d.nsf_m, d.chi_m, g.qext,
                                                        (float *)g.q3, nc, d.G, g.Gp);
    dg_check_launch();
}

void launch_dg_finalize(const DevProblem &d, const DevDG &g, double *phi_internal, double *phi_user, double *partials,
                        hipStream_t s) {
    k_dg_finalize<<<kReduceBlocks, 256, 0, s>>>(g.tally, d.V, g.hV, g.mat3, d.nsf_m, d.user_of, phi_internal, phi_user,
                                                partials, g.Nz, d.R, d.G, g.Gp);
    dg_check_launch();
}

void launch_dg_fission_partials(const DevProblem &d, const DevDG &g, const double *phi, double *partials, hipStream_t s) {
    k_dg_fission_partials<<<kReduceBlocks, 256, 0, s>>>(phi, g.hV, g.mat3, d.nsf_m, partials, (int64_t)g.Nz * d.R, d.G);
    dg_check_launch();
}

void launch_dg_norm_residual(const DevProblem &d, const DevDG &g, double *phi_new, const double *phi_old, double *partials,
                             hipStream_t s) {
    k_dg_norm_residual<<<kReduceBlocks, 256, 0, s>>>(phi_new, phi_old, g.hV, d.scal, partials, (int64_t)g.Nz * d.R, d.G);
    k_dg_residual<<<1, 256, 0, s>>>(partials, kReduceBlocks, d.scal);
    dg_check_launch();
}

void launch_dg_cold_flux(const DevDG &g, double *phi, int64_t n_cells, hipStream_t s) {
    (void)g;
    k_dg_cold<<<grid_for(n_cells), 256, 0, s>>>(phi, n_cells);
    dg_check_launch();
}

void launch_dg_permute(const DevProblem &d, const DevDG &g, const double *src, double *dst, int to_user, hipStream_t s) {
    const int64_t n = (int64_t)g.Nz * d.R * d.G * 2;
    k_dg_permute<<<grid_for(n), 256, 0, s>>>(src, dst, d.user_of, g.Nz, d.R, d.G, to_user);
    dg_check_launch();
}

}  // namespace moc
