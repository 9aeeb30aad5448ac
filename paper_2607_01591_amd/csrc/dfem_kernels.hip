// HIP kernels of libmoc's DFEM-SN solver for gfx950 (CDNA4): one sweep step (one
// dependency level of every direction), source, finalisation and the FP64 reductions of
// the power iteration.
//
// Local system of element e, direction Omega, group g (Sec. 2.2, Eq. DFEM_parts with the
// upwind flux of Eq. DFEM_upwind), modal basis u = (1, (x - x_c)/L, (y - y_c)/L):
//   A_ji = Sigma_t M_ji - (Omega . grad u_j) int u_i + sum_{outflow faces} (Omega . n) E_f,ji
//   b_j  = sum_i M_ji q_i - sum_{inflow faces} (Omega . n) int_f u_j psi_up
// where int u_i = area delta_i0 (the slopes have zero mean), E_f the face matrix of the
// element's own basis and, for an interior inflow face, int_f u_j psi_up = C_f psi_nb with
// the coupling matrix C_f of the two bases on the shared face.
#include <cmath>

#include "dfem_kernels.h"
#include "moc.h"
#include "moc_internal.h"

namespace moc {

static constexpr double kFourPiSn = 12.566370614359172953850573533118;


// Where the local solve reads its data: straight from the global arrays (level schedule)
// or from a tile task's copy in LDS (tiled schedule). Both present the same values, so the
// solve below does the same arithmetic in the same order for either.
template <typename Real, int kG = 0> struct SnGlobalSrc {
    const SnStepArgs &a;
    int64_t k;
    int e, d;
    __device__ SnGlobalSrc(const SnStepArgs &a_, int64_t k_) : a(a_), k(k_), e(a_.task_e[k_]), d(a_.task_d[k_]) {}
    __device__ const Real *mass() const { return reinterpret_cast<const Real *>(a.mass) + (int64_t)e * 6; }
    __device__ Real gradw() const { return reinterpret_cast<const Real *>(a.gradw)[e]; }
    __device__ const Real *nrm(int f) const { return reinterpret_cast<const Real *>(a.nrm) + ((int64_t)e * 3 + f) * 2; }
    __device__ const Real *fmass(int f) const { return reinterpret_cast<const Real *>(a.fmass) + ((int64_t)e * 3 + f) * 6; }
    __device__ const Real *fcpl(int f) const { return reinterpret_cast<const Real *>(a.fcpl) + ((int64_t)e * 3 + f) * 9; }
    __device__ Real sigt(int g) const { return reinterpret_cast<const Real *>(a.sigt)[(int64_t)e * ng() + g]; }
    __device__ const Real *q(int g) const { return reinterpret_cast<const Real *>(a.q) + ((int64_t)e * ng() + g) * 3; }
    __device__ const Real *dir() const { return reinterpret_cast<const Real *>(a.dirs) + 3 * d; }
    __device__ int code(int f) const { return a.inflow[3 * k + f]; }
    __device__ int bwrite(int f) const { return a.bwrite[3 * k + f]; }
    __device__ int slot() const { return a.task_slot[k]; }
    // upstream flux of inflow code c >= 0 (a storage slot) or c <= -4 (boundary entry)
    __device__ const Real *upstream(int c, int g) const {
        return c >= 0 ? reinterpret_cast<const Real *>(a.psi) + ((int64_t)c * ng() + g) * 3
                      : reinterpret_cast<const Real *>(a.bnd_in) + ((int64_t)(-4 - c) * ng() + g) * 3;
    }
    __device__ void store_local(int, int, const Real *) const {}
    __device__ int ng() const { return kG > 0 ? kG : a.G; }
};

// Size of the face block a direction group needs for inflow code c: the coupling matrix
// (9) for an interior inflow, the face matrix (6) for an outflow or a reflective inflow,
// nothing for a vacuum inflow.
__device__ __forceinline__ int sn_face_reals(int c) { return c == kSnVacuum ? 0 : (c >= 0 ? 9 : 6); }

// LDS copy of one tile task: element data per item [item][el_stride] (mass 6, gradw 1,
// normals 6, then per face only the matrix the item's direction group uses), (Sigma_t, q)
// [tile element][G][4], item records [item][kSnRecInts], the fluxes entering from other
// tiles or the boundary [entry][G][3], the direction group's directions, and the tile's
// own fluxes in compressed slots [slot][tgroup][G][3]. Polar direction pp of an item reads
// its record with the offsets of the record's layout (entries, boundary writes and storage
// slots of the item's directions are consecutive).
template <typename Real, int kG, int kTG> struct SnLdsSrc {
    const SnStepArgs &a;
    const Real *el, *sq, *ext, *dirs;
    Real *psi_l;
    const int *tk;
    int it, loc, pp;
    int eo, fo1, fo2;    // the item's element block and the offsets of its face 1 and 2 blocks
    __device__ int ng() const { return kG > 0 ? kG : a.G; }
    __device__ int ntg() const { return kTG > 0 ? kTG : a.tgroup; }
    __device__ const Real *mass() const { return el + eo; }
    __device__ Real gradw() const { return el[eo + 6]; }
    __device__ const Real *nrm(int f) const { return el + eo + 7 + 2 * f; }
    __device__ const Real *face(int f) const { return el + eo + 13 + (f == 0 ? 0 : f == 1 ? fo1 : fo2); }
    __device__ const Real *fmass(int f) const { return face(f); }
    __device__ const Real *fcpl(int f) const { return face(f); }
    __device__ Real sigt(int g) const { return sq[(loc * ng() + g) * 4]; }
    __device__ const Real *q(int g) const { return sq + (loc * ng() + g) * 4 + 1; }
    __device__ const Real *dir() const { return dirs + 3 * pp; }
    __device__ int code(int f) const {
        const int c = tk[it * kSnRecInts + 2 + f];
        if (c <= -4) return c - pp;
        return (c >= 0 && !(c & kSnLocalFlag)) ? c + pp : c;
    }
    __device__ int bwrite(int f) const {
        const int w = tk[it * kSnRecInts + 5 + f];
        return w >= 0 ? w + pp : -1;
    }
    __device__ int slot() const {
        const int sl = tk[it * kSnRecInts + 8];
        return sl >= 0 ? sl + pp : -1;
    }
    // c >= 0 with kSnLocalFlag: the tile's own flux of that element; c >= 0 with
    // kSnExtFlag: staged entry (another tile's slot); c <= -4: staged entry -4 - c (the
    // boundary buffer)
    __device__ const Real *upstream(int c, int g) const {
        if (c < 0) return ext + ((-4 - c) * ng() + g) * 3;
        return (c & kSnLocalFlag) ? psi_l + (((c & ~kSnLocalFlag) * ntg() + pp) * ng() + g) * 3
                                  : ext + ((c & ~kSnExtFlag) * ng() + g) * 3;
    }
    __device__ void store_local(int g, int, const Real *x) const {
        const int ls = tk[it * kSnRecInts + 1];
        if (ls < 0) return;   // read by no element of the tile
        Real *pl = psi_l + ((ls * ntg() + pp) * ng() + g) * 3;
        pl[0] = x[0];
        pl[1] = x[1];
        pl[2] = x[2];
    }
};

// The local solve of one task (element, direction) for group g, shared by both
// schedules: A = Sigma_t M - (Omega . grad u) int u + outflow face terms, b = M q -
// inflow face terms, solved in closed form. Writes psi to the task's
// storage slot (slot >= 0), to the boundary buffer on reflective outflow faces and, tiled,
// to the tile's LDS copy; returns w psi in contrib.
template <typename Real, typename Src>
__device__ __forceinline__ void sn_task(const SnStepArgs &a, const Src &S, int g, double (&contrib)[3]) {
    const int G = S.ng();
    Real *__restrict__ psi = reinterpret_cast<Real *>(a.psi);
    Real *__restrict__ bnd_out = reinterpret_cast<Real *>(a.bnd_out);
    const Real *dr = S.dir();
    const Real ox = dr[0], oy = dr[1], wd = dr[2];
    const Real st = S.sigt(g);
    const Real *m = S.mass();
    const Real M[9] = {m[0], m[1], m[2], m[1], m[3], m[4], m[2], m[4], m[5]};
    Real A[9], b[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i] = st * M[i];
    const Real gw = S.gradw();
    A[3] -= ox * gw;
    A[6] -= oy * gw;
    const Real *qe = S.q(g);
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = M[3 * j] * qe[0] + M[3 * j + 1] * qe[1] + M[3 * j + 2] * qe[2];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int code = S.code(f);
        if (code == kSnVacuum) continue;
        const Real *nf = S.nrm(f);
        const Real on = ox * nf[0] + oy * nf[1];
        const Real *E = S.fmass(f);
        if (code == kSnOutflow) {
            const Real Ef[9] = {E[0], E[1], E[2], E[1], E[3], E[4], E[2], E[4], E[5]};
#pragma unroll
            for (int i = 0; i < 9; ++i) A[i] += on * Ef[i];
        } else if (code >= 0) {
            // interior inflow: upstream flux through the coupling matrix
            const Real *pu = S.upstream(code, g);
            const Real u0 = pu[0], u1 = pu[1], u2 = pu[2];
            const Real *C = S.fcpl(f);
#pragma unroll
            for (int j = 0; j < 3; ++j) b[j] -= on * (C[3 * j] * u0 + C[3 * j + 1] * u1 + C[3 * j + 2] * u2);
        } else {
            // reflective boundary inflow (code <= -4) through the element's own face matrix
            const Real *pb = S.upstream(code, g);
            const Real u0 = pb[0], u1 = pb[1], u2 = pb[2];
            const Real Ef[9] = {E[0], E[1], E[2], E[1], E[3], E[4], E[2], E[4], E[5]};
#pragma unroll
            for (int j = 0; j < 3; ++j) b[j] -= on * (Ef[3 * j] * u0 + Ef[3 * j + 1] * u1 + Ef[3 * j + 2] * u2);
        }
    }
    // x = adj(A) b / det(A): the cofactors C_ij of A, det along the first row, one
    // division. No pivoting is needed: integrating the streaming term by parts gives
    // u^T A u = Sigma_t |u|^2 + 1/2 sum over faces of int |Omega . n| u^2 > 0, so the
    // symmetric part of A is positive definite and det(A) > 0.
    const Real c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    const Real c10 = A[2] * A[7] - A[1] * A[8], c11 = A[0] * A[8] - A[2] * A[6], c12 = A[1] * A[6] - A[0] * A[7];
    const Real c20 = A[1] * A[5] - A[2] * A[4], c21 = A[2] * A[3] - A[0] * A[5], c22 = A[0] * A[4] - A[1] * A[3];
    const Real rdet = Real(1) / (A[0] * c00 + A[1] * c01 + A[2] * c02);
    Real x[3];
    x[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) * rdet;
    x[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) * rdet;
    x[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * rdet;
    const int sl = S.slot();
    if (sl >= 0) {
        Real *ps = psi + ((int64_t)sl * G + g) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) ps[i] = x[i];
    }
    S.store_local(g, 0, x);
#pragma unroll
    for (int i = 0; i < 3; ++i) contrib[i] = (double)(wd * x[i]);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int wi = S.bwrite(f);
        if (wi >= 0) {
            Real *o = bnd_out + ((int64_t)wi * G + g) * 3;
            o[0] = x[0];
            o[1] = x[1];
            o[2] = x[2];
        }
    }
}

// sums each run of TG lanes onto its first lane, which stores it at run_acc row r
// (direction group, element); every lane of the wavefront takes part in the shuffles (idle
// lanes carry zeros, and a run never crosses a wavefront)
template <typename Real, int kG = 0, int kTG = 0>
__device__ __forceinline__ void sn_store_run(const SnStepArgs &a, int pp, bool valid, int64_t r, int g, double (&contrib)[3]) {
    const int TG = kTG > 0 ? kTG : a.tgroup;
    const int G = kG > 0 ? kG : a.G;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double sum = contrib[i];
        for (int j = 1; j < TG; ++j) {
            const double v = __shfl_down(contrib[i], j, 64);
            if (pp + j < TG) sum += v;
        }
        contrib[i] = sum;
    }
    if (valid && pp == 0) {
        Real *ra = reinterpret_cast<Real *>(a.run_acc) + (r * G + g) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) ra[i] = (Real)contrib[i];
    }
}

// One sweep step of the level schedule: every (element, direction) task of one dependency
// level, for every group, one thread per (task, group). A run of tgroup consecutive tasks
// (the polar directions of one element and azimuth) sits on adjacent lanes of one
// wavefront for each group (64 / tgroup runs per wavefront, the remaining lanes idle), so
// the lanes of a run read the same element data and their contributions to the element's
// scalar-flux moments are summed across the run with wavefront shuffles and stored once
// per run (no atomics; k_sn_gather adds them after the last level). The upstream elements
// of a task belong to earlier levels, whose angular fluxes sit in their storage slots.
template <typename Real, int kG, int kTG> __global__ void __launch_bounds__(256) k_sn_step(SnStepArgs a) {
    const int G = kG > 0 ? kG : a.G, TG = kTG > 0 ? kTG : a.tgroup;
    const int runs_per_wave = 64 / TG;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int pp = lane % TG;
    const int64_t run = wave * runs_per_wave + lane / TG;
    const int64_t nrun = (a.k1 - a.k0) / TG * G;
    const bool valid = lane < runs_per_wave * TG && run < nrun;
    double contrib[3] = {0.0, 0.0, 0.0};
    const int64_t kg = run / G;
    const int g = int(run - kg * G);
    const int64_t k = a.k0 + kg * TG + pp;
    int64_t r = 0;
    if (valid) {
        const SnGlobalSrc<Real, kG> S(a, k);
        sn_task<Real>(a, S, g, contrib);
        r = (int64_t)(S.d / TG) * a.T + S.e;
    }
    sn_store_run<Real, kG, kTG>(a, pp, valid, r, g, contrib);
}

// Tiled schedule: one block per (tile, direction group) of one tile level. The block first
// copies everything its tasks read into LDS in one round of independent loads (element
// data, Sigma_t and q of the tile's elements, the item records, the fluxes entering from
// earlier tiles and from the boundary, the directions), then walks the tile's own
// dependency levels with a workgroup barrier between two of them, reading only LDS: the
// tile's own fluxes stay there in slots reused once their last reader in the tile is done,
// fluxes read by a later tile go to storage slots.
template <typename Real, int kG, int kTG>
__global__ void __launch_bounds__(256) k_sn_tile(SnStepArgs a, SnTileArgs t) {
    extern __shared__ __align__(16) unsigned char sn_lds[];
    Real *psi_l = reinterpret_cast<Real *>(sn_lds + t.lds_off[kSnLdsPsi]);
    Real *el = reinterpret_cast<Real *>(sn_lds + t.lds_off[kSnLdsElem]);
    Real *sq = reinterpret_cast<Real *>(sn_lds + t.lds_off[kSnLdsSq]);
    Real *ext = reinterpret_cast<Real *>(sn_lds + t.lds_off[kSnLdsExt]);
    Real *dl = reinterpret_cast<Real *>(sn_lds + t.lds_off[kSnLdsDir]);
    int *tk = reinterpret_cast<int *>(sn_lds + t.lds_off[kSnLdsTask]);
    int *eg = reinterpret_cast<int *>(sn_lds + t.lds_off[kSnLdsElemId]);
    int *fo = reinterpret_cast<int *>(sn_lds + t.lds_off[kSnLdsFine]);
    const int G = kG > 0 ? kG : a.G, TG = kTG > 0 ? kTG : a.tgroup;
    const int64_t tt = t.tt0 + blockIdx.x;
    const int64_t ibase = t.tt_task[tt] / TG;
    const int nit = int(t.tt_task[tt + 1] / TG - ibase);
    const int tile = t.tt_tile[tt], dg = t.tt_dg[tt];
    const int toff = t.tile_off[tile], nel = t.tile_off[tile + 1] - toff;
    const int x0 = t.ext_off[tt], nx = t.ext_off[tt + 1] - x0;
    const int f0 = t.tt_fine[tt], nf = t.tt_fine[tt + 1] - f0;   // nf - 1 levels
    const Real *__restrict__ gmass = reinterpret_cast<const Real *>(a.mass);
    const Real *__restrict__ ggw = reinterpret_cast<const Real *>(a.gradw);
    const Real *__restrict__ gnrm = reinterpret_cast<const Real *>(a.nrm);
    const Real *__restrict__ gfm = reinterpret_cast<const Real *>(a.fmass);
    const Real *__restrict__ gfc = reinterpret_cast<const Real *>(a.fcpl);
    const Real *__restrict__ gst = reinterpret_cast<const Real *>(a.sigt);
    const Real *__restrict__ gq = reinterpret_cast<const Real *>(a.q);
    const Real *__restrict__ gpsi = reinterpret_cast<const Real *>(a.psi);
    const Real *__restrict__ gbnd = reinterpret_cast<const Real *>(a.bnd_in);
    const Real *__restrict__ gdir = reinterpret_cast<const Real *>(a.dirs);
    // ---- stage
    const int els = t.el_stride;
    for (int i = threadIdx.x; i < nit; i += blockDim.x) {   // one thread per item's element block
        const int *r = t.rec + (ibase + i) * kSnRecInts;
        const int64_t e = t.tile_elems[toff + r[0]];
        Real *o = el + i * els;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = gmass[e * 6 + c];
        o[6] = ggw[e];
#pragma unroll
        for (int c = 0; c < 6; ++c) o[7 + c] = gnrm[e * 6 + c];
        int off = 13;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int code = r[2 + f];
            if (code == kSnVacuum) continue;
            if (code >= 0) {
#pragma unroll
                for (int c = 0; c < 9; ++c) o[off + c] = gfc[e * 27 + f * 9 + c];
                off += 9;
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) o[off + c] = gfm[e * 18 + f * 6 + c];
                off += 6;
            }
        }
    }
    for (int i = threadIdx.x; i < nel * G; i += blockDim.x) {
        const int l = i / G, g = i - l * G;
        const int64_t e = t.tile_elems[toff + l];
        sq[i * 4] = gst[e * G + g];
        sq[i * 4 + 1] = gq[(e * G + g) * 3];
        sq[i * 4 + 2] = gq[(e * G + g) * 3 + 1];
        sq[i * 4 + 3] = gq[(e * G + g) * 3 + 2];
    }
    for (int i = threadIdx.x; i < nit * kSnRecInts; i += blockDim.x) tk[i] = t.rec[ibase * kSnRecInts + i];
    for (int i = threadIdx.x; i < nx * G; i += blockDim.x) {
        const int j = i / G, g = i - j * G;
        const int src = t.ext_src[x0 + j];
        const Real *p = src >= 0 ? gpsi + ((int64_t)src * G + g) * 3 : gbnd + ((int64_t)(-4 - src) * G + g) * 3;
        ext[i * 3] = p[0];
        ext[i * 3 + 1] = p[1];
        ext[i * 3 + 2] = p[2];
    }
    for (int i = threadIdx.x; i < TG * 3; i += blockDim.x) dl[i] = gdir[(int64_t)dg * TG * 3 + i];
    for (int i = threadIdx.x; i < nel; i += blockDim.x) eg[i] = t.tile_elems[toff + i];
    for (int i = threadIdx.x; i < nf; i += blockDim.x) fo[i] = t.fine_off[f0 + i];
    __syncthreads();
    // ---- the tile's levels
    const int runs_per_wave = 64 / TG;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int pp = lane % TG;
    SnLdsSrc<Real, kG, kTG> S{a, el, sq, ext, dl, psi_l, tk, 0, 0, pp, 0, 0, 0};
    for (int fl = 0; fl + 1 < nf; ++fl) {
        const int k0 = fo[fl], nrun = (fo[fl + 1] - k0) / TG * G;
        for (int r0 = wave * runs_per_wave; r0 < nrun; r0 += nwave * runs_per_wave) {
            const int run = r0 + lane / TG;
            const bool valid = lane < runs_per_wave * TG && run < nrun;
            double contrib[3] = {0.0, 0.0, 0.0};
            const int kg = run / G;
            const int g = run - kg * G;
            int64_t r = 0;
            if (valid) {
                S.it = k0 / TG + kg;
                S.loc = tk[S.it * kSnRecInts];
                S.eo = S.it * els;
                S.fo1 = sn_face_reals(tk[S.it * kSnRecInts + 2]);
                S.fo2 = S.fo1 + sn_face_reals(tk[S.it * kSnRecInts + 3]);
                sn_task<Real>(a, S, g, contrib);
                r = (int64_t)dg * a.T + eg[S.loc];
            }
            sn_store_run<Real, kG, kTG>(a, pp, valid, r, g, contrib);
        }
        __syncthreads();   // this level's LDS fluxes before the next level reads them
    }
}

// Scalar-flux moments of every element: the sum over the direction groups, in direction
// order (the same order for both schedules), one thread per (element, group, moment);
// run_acc is [direction group][T][G][3], so each term of the sum is a coalesced read.
template <typename Real>
__global__ void k_sn_gather(const Real *__restrict__ run_acc, double *__restrict__ phi_acc, int T, int G, int ndg) {
    const int64_t n = (int64_t)T * G * 3;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < ndg; ++j) acc += (double)run_acc[(int64_t)j * n + t];
        phi_acc[t] = acc;
    }
}

// q = s / (4 pi) from a caller's emission moments
template <typename Real> __global__ void k_sn_prep(const double *__restrict__ src, Real *__restrict__ q, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        q[i] = (Real)(src[i] / kFourPiSn);
}

// Emission moments (Eq. MGNTE, isotropic): s_i = sum_g' Sigma_s,g'->g phi_i,g'
// + chi_g F_i / k (+ external), per modal coefficient i; q = s / (4 pi). One thread per
// (element, group).
template <typename Real>
__global__ void k_sn_source(const double *__restrict__ phi, const double *__restrict__ scal, const int *__restrict__ mat,
                            const double *__restrict__ sigs_m, const double *__restrict__ nsf_m,
                            const double *__restrict__ chi_m, const double *__restrict__ qext, Real *__restrict__ q, int T,
                            int G) {
    const double inv_k = 1.0 / scal[kSnK];
    const int64_t n = (int64_t)T * G;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / G;
        const int g = int(t - e * G);
        const int m = mat[e];
        const double *ph = phi + e * G * 3;
        double F[3] = {0, 0, 0}, s[3] = {0, 0, 0};
        for (int gp = 0; gp < G; ++gp) {
            const double nf = nsf_m[m * G + gp], sc = sigs_m[((int64_t)m * G + gp) * G + g];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                F[i] += nf * ph[3 * gp + i];
                s[i] += sc * ph[3 * gp + i];
            }
        }
        const double ch = chi_m[m * G + g] * inv_k;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double v = s[i] + ch * F[i];
            if (qext) v += qext[t * 3 + i];
            q[t * 3 + i] = (Real)(v / kFourPiSn);
        }
    }
}

__device__ __forceinline__ double sn_block_sum(double v, double *sh) {
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

// phi = accumulated moments, to the internal flux (with partials of sum area nuSigma_f
// phi_0) or to a caller's buffer
__global__ void k_sn_finalize(const double *__restrict__ acc, const double *__restrict__ area, const int *__restrict__ mat,
                              const double *__restrict__ nsf_m, double *__restrict__ phi_internal,
                              double *__restrict__ phi_user, double *__restrict__ partials, int T, int G) {
    __shared__ double sh[16];
    double f = 0.0;
    const int64_t n = (int64_t)T * G;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / G;
        const int g = int(t - e * G);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double v = acc[t * 3 + i];
            if (phi_internal) phi_internal[t * 3 + i] = v;
            if (phi_user) phi_user[t * 3 + i] = v;
        }
        f += area[e] * nsf_m[mat[e] * G + g] * acc[t * 3];
    }
    if (partials) {
        const double s = sn_block_sum(f, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

__global__ void k_sn_fission_partials(const double *__restrict__ phi, const double *__restrict__ area,
                                      const int *__restrict__ mat, const double *__restrict__ nsf_m,
                                      double *__restrict__ partials, int T, int G) {
    __shared__ double sh[16];
    double f = 0.0;
    const int64_t n = (int64_t)T * G;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / G;
        const int g = int(t - e * G);
        f += area[e] * nsf_m[mat[e] * G + g] * phi[t * 3];
    }
    const double s = sn_block_sum(f, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Single block. mode 0: initial normalisation; 1: k <- k sum (old sum = 1); 2: fixed source.
__global__ void k_sn_eigen_update(const double *__restrict__ partials, int nblk, double *__restrict__ scal, int mode) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partials[i];
    const double s = sn_block_sum(acc, sh);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            scal[kSnF] = 1.0 / s;
        } else if (mode == 1) {
            scal[kSnKPrev] = scal[kSnK];
            scal[kSnK] = scal[kSnK] * s;
            scal[kSnF] = 1.0 / s;
        } else {
            scal[kSnKPrev] = scal[kSnK];
            scal[kSnF] = 1.0;
        }
    }
}

// phi_new *= f; partials of the mass-weighted squared norms of the change and of the new
// field (the L2 norm of the linear field on each element and group)
__global__ void k_sn_norm_residual(double *__restrict__ phi_new, const double *__restrict__ phi_old,
                                   const double *__restrict__ massd, const double *__restrict__ scal,
                                   double *__restrict__ partials, int T, int G) {
    __shared__ double sh[16];
    const double f = scal[kSnF];
    double num = 0.0, den = 0.0;
    const int64_t n = (int64_t)T * G;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / G;
        const double *Me = massd + e * 9;
        double x[3], dlt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = phi_new[t * 3 + i] * f;
            phi_new[t * 3 + i] = x[i];
            dlt[i] = x[i] - phi_old[t * 3 + i];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                num += dlt[j] * Me[3 * j + i] * dlt[i];
                den += x[j] * Me[3 * j + i] * x[i];
            }
    }
    const double sa = sn_block_sum(num, sh);
    const double sb = sn_block_sum(den, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sa;
        partials[2 * blockIdx.x + 1] = sb;
    }
}

__global__ void k_sn_residual(const double *__restrict__ partials, int nblk, double *__restrict__ scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    const double sa = sn_block_sum(a, sh);
    const double sb = sn_block_sum(b, sh);
    if (threadIdx.x == 0) {
        scal[kSnRes] = sb > 0 ? sqrt(sa / sb) : 0.0;
        scal[kSnDk] = fabs(scal[kSnK] - scal[kSnKPrev]);
    }
}

template <typename T> __global__ void k_sn_fill(T *__restrict__ p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
template <typename T> __global__ void k_sn_scale(T *__restrict__ p, int64_t n, const double *__restrict__ f) {
    const T s = (T)(*f);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] *= s;
}
__global__ void k_sn_cold(double *__restrict__ phi, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        phi[i] = (i % 3 == 0) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- launchers
static void sn_check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(MOC_EHIP, hipGetErrorString(e));
}

static int sn_grid(int64_t n, int block = 256, int cap = 8192) {
    const int64_t b = (n + block - 1) / block;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

void launch_sn_step(const SnStepArgs &a, int precision, hipStream_t s) {
    // exactly one thread per (task, group) slot: waves of 64 / tgroup runs of tgroup lanes
    const int64_t nrun = (a.k1 - a.k0) / a.tgroup * a.G;
    if (nrun <= 0) return;
    const int64_t runs_per_wave = 64 / a.tgroup;
    const int64_t waves = (nrun + runs_per_wave - 1) / runs_per_wave;
    const int64_t blocks = (waves + 3) / 4;
    const bool g7p3 = a.G == 7 && a.tgroup == 3;   // the usual shape, sizes known to the compiler
    if (precision == MOC_PREC_F64) {
        if (g7p3) k_sn_step<double, 7, 3><<<(unsigned)blocks, 256, 0, s>>>(a);
        else k_sn_step<double, 0, 0><<<(unsigned)blocks, 256, 0, s>>>(a);
    } else {
        if (g7p3) k_sn_step<float, 7, 3><<<(unsigned)blocks, 256, 0, s>>>(a);
        else k_sn_step<float, 0, 0><<<(unsigned)blocks, 256, 0, s>>>(a);
    }
    sn_check_launch();
}

void launch_sn_gather(const DevSN &d, hipStream_t s) {
    const int64_t n = (int64_t)d.T * d.G * 3;
    if (d.precision == MOC_PREC_F64)
        k_sn_gather<double><<<sn_grid(n), 256, 0, s>>>((const double *)d.run_acc, d.phi_acc, d.T, d.G, d.ndg);
    else
        k_sn_gather<float><<<sn_grid(n), 256, 0, s>>>((const float *)d.run_acc, d.phi_acc, d.T, d.G, d.ndg);
    sn_check_launch();
}

void launch_sn_tile(const SnStepArgs &a, const SnTileArgs &t, int nblocks, size_t lds_bytes, int precision, hipStream_t s) {
    if (nblocks <= 0) return;
    // the usual shape (7 groups, 3 polar directions per azimuth) with its sizes known to the
    // compiler, every other shape through the general instance
    const bool g7p3 = a.G == 7 && a.tgroup == 3;
    if (precision == MOC_PREC_F64) {
        if (g7p3) k_sn_tile<double, 7, 3><<<(unsigned)nblocks, 256, lds_bytes, s>>>(a, t);
        else k_sn_tile<double, 0, 0><<<(unsigned)nblocks, 256, lds_bytes, s>>>(a, t);
    } else {
        if (g7p3) k_sn_tile<float, 7, 3><<<(unsigned)nblocks, 256, lds_bytes, s>>>(a, t);
        else k_sn_tile<float, 0, 0><<<(unsigned)nblocks, 256, lds_bytes, s>>>(a, t);
    }
    sn_check_launch();
}

void launch_sn_prep_user(const DevSN &d, const double *src, hipStream_t s) {
    const int64_t n = (int64_t)d.T * d.G * 3;
    if (d.precision == MOC_PREC_F64)
        k_sn_prep<double><<<sn_grid(n), 256, 0, s>>>(src, (double *)d.q, n);
    else
        k_sn_prep<float><<<sn_grid(n), 256, 0, s>>>(src, (float *)d.q, n);
    sn_check_launch();
}

void launch_sn_source(const DevSN &d, const double *phi, hipStream_t s) {
    const int64_t n = (int64_t)d.T * d.G;
    if (d.precision == MOC_PREC_F64)
        k_sn_source<double><<<sn_grid(n), 256, 0, s>>>(phi, d.scal, d.mat, d.sigs_m, d.nsf_m, d.chi_m, d.qext,
                                                       (double *)d.q, d.T, d.G);
    else
        k_sn_source<float><<<sn_grid(n), 256, 0, s>>>(phi, d.scal, d.mat, d.sigs_m, d.nsf_m, d.chi_m, d.qext,
                                                      (float *)d.q, d.T, d.G);
    sn_check_launch();
}

void launch_sn_finalize(const DevSN &d, double *phi_internal, double *phi_user, double *partials, hipStream_t s) {
    k_sn_finalize<<<kSnReduceBlocks, 256, 0, s>>>(d.phi_acc, d.area, d.mat, d.nsf_m, phi_internal, phi_user, partials,
                                                  d.T, d.G);
    sn_check_launch();
}

void launch_sn_fission_partials(const DevSN &d, const double *phi, hipStream_t s) {
    k_sn_fission_partials<<<kSnReduceBlocks, 256, 0, s>>>(phi, d.area, d.mat, d.nsf_m, d.partials, d.T, d.G);
    sn_check_launch();
}

void launch_sn_eigen_update(const DevSN &d, int mode, hipStream_t s) {
    k_sn_eigen_update<<<1, 256, 0, s>>>(d.partials, kSnReduceBlocks, d.scal, mode);
    sn_check_launch();
}

void launch_sn_norm_residual(const DevSN &d, double *phi_new, const double *phi_old, hipStream_t s) {
    k_sn_norm_residual<<<kSnReduceBlocks, 256, 0, s>>>(phi_new, phi_old, d.massd, d.scal, d.partials, d.T, d.G);
    k_sn_residual<<<1, 256, 0, s>>>(d.partials, kSnReduceBlocks, d.scal);
    sn_check_launch();
}

void launch_sn_fill(void *p, int64_t n, int precision, hipStream_t s) {
    if (n <= 0) return;
    if (precision == MOC_PREC_F64)
        k_sn_fill<double><<<sn_grid(n), 256, 0, s>>>((double *)p, n, 0.0);
    else
        k_sn_fill<float><<<sn_grid(n), 256, 0, s>>>((float *)p, n, 0.0f);
    sn_check_launch();
}

void launch_sn_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    k_sn_fill<double><<<sn_grid(n), 256, 0, s>>>(p, n, v);
    sn_check_launch();
}

void launch_sn_scale(void *p, int64_t n, int precision, const double *f, hipStream_t s) {
    if (n <= 0) return;
    if (precision == MOC_PREC_F64)
        k_sn_scale<double><<<sn_grid(n), 256, 0, s>>>((double *)p, n, f);
    else
        k_sn_scale<float><<<sn_grid(n), 256, 0, s>>>((float *)p, n, f);
    sn_check_launch();
}

void launch_sn_scale_f64(double *p, int64_t n, const double *f, hipStream_t s) {
    if (n <= 0) return;
    k_sn_scale<double><<<sn_grid(n), 256, 0, s>>>(p, n, f);
    sn_check_launch();
}

void launch_sn_cold(double *phi, int64_t n, hipStream_t s) {
    k_sn_cold<<<sn_grid(n), 256, 0, s>>>(phi, n);
    sn_check_launch();
}

}  // namespace moc
