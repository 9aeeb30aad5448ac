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

// One sweep step: every (element, direction) task of one dependency level, for every
// group, one thread per (task, group). A run of tgroup consecutive tasks (the polar
// directions of one element and azimuth) sits on adjacent lanes of one wavefront for each
// group (64 / tgroup runs per wavefront, the remaining lanes idle), so the lanes of a run
// read the same element data and their contributions to the element's scalar-flux moments
// are summed across the run with wavefront shuffles and stored once per run (no atomics;
// k_sn_gather adds the runs of each element after the last level). The upstream elements
// of a task belong to earlier levels, whose angular fluxes sit in their storage slots.
template <typename Real> __global__ void __launch_bounds__(256) k_sn_step(SnStepArgs a) {
    const int G = a.G, TG = a.tgroup;
    const int runs_per_wave = 64 / TG;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int pp = lane % TG;
    const int64_t run = wave * runs_per_wave + lane / TG;
    const int64_t nrun = (a.k1 - a.k0) / TG * G;
    const bool valid = lane < runs_per_wave * TG && run < nrun;
    const Real *__restrict__ mass = reinterpret_cast<const Real *>(a.mass);
    const Real *__restrict__ fmass = reinterpret_cast<const Real *>(a.fmass);
    const Real *__restrict__ fcpl = reinterpret_cast<const Real *>(a.fcpl);
    const Real *__restrict__ nrm = reinterpret_cast<const Real *>(a.nrm);
    const Real *__restrict__ gradw = reinterpret_cast<const Real *>(a.gradw);
    const Real *__restrict__ sigt = reinterpret_cast<const Real *>(a.sigt);
    const Real *__restrict__ dirs = reinterpret_cast<const Real *>(a.dirs);
    const Real *__restrict__ q = reinterpret_cast<const Real *>(a.q);
    Real *__restrict__ psi = reinterpret_cast<Real *>(a.psi);
    const Real *__restrict__ bnd_in = reinterpret_cast<const Real *>(a.bnd_in);
    Real *__restrict__ bnd_out = reinterpret_cast<Real *>(a.bnd_out);
    double contrib[3] = {0.0, 0.0, 0.0};
    const int64_t kg = run / G;
    const int g = int(run - kg * G);
    if (valid) {
        const int64_t k = a.k0 + kg * TG + pp;
        const int e = a.task_e[k];
        const int d = a.task_d[k];
        const Real ox = dirs[3 * d], oy = dirs[3 * d + 1], wd = dirs[3 * d + 2];
        const Real st = sigt[(int64_t)e * G + g];
        const Real *m = mass + (int64_t)e * 6;
        const Real M[9] = {m[0], m[1], m[2], m[1], m[3], m[4], m[2], m[4], m[5]};
        Real A[9], b[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) A[i] = st * M[i];
        const Real gw = gradw[e];
        A[3] -= ox * gw;
        A[6] -= oy * gw;
        const Real *qe = q + ((int64_t)e * G + g) * 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) b[j] = M[3 * j] * qe[0] + M[3 * j + 1] * qe[1] + M[3 * j + 2] * qe[2];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int code = a.inflow[3 * k + f];
            if (code == kSnVacuum) continue;
            const Real on = ox * nrm[((int64_t)e * 3 + f) * 2] + oy * nrm[((int64_t)e * 3 + f) * 2 + 1];
            const Real *E = fmass + ((int64_t)e * 3 + f) * 6;
            if (code == kSnOutflow) {
                const Real Ef[9] = {E[0], E[1], E[2], E[1], E[3], E[4], E[2], E[4], E[5]};
#pragma unroll
                for (int i = 0; i < 9; ++i) A[i] += on * Ef[i];
            } else if (code >= 0) {
                const Real *pu = psi + ((int64_t)code * G + g) * 3;
                const Real u0 = pu[0], u1 = pu[1], u2 = pu[2];
                const Real *C = fcpl + ((int64_t)e * 3 + f) * 9;
#pragma unroll
                for (int j = 0; j < 3; ++j) b[j] -= on * (C[3 * j] * u0 + C[3 * j + 1] * u1 + C[3 * j + 2] * u2);
            } else {
                const Real *pb = bnd_in + ((int64_t)(-4 - code) * G + g) * 3;
                const Real u0 = pb[0], u1 = pb[1], u2 = pb[2];
                const Real Ef[9] = {E[0], E[1], E[2], E[1], E[3], E[4], E[2], E[4], E[5]};
#pragma unroll
                for (int j = 0; j < 3; ++j) b[j] -= on * (Ef[3 * j] * u0 + Ef[3 * j + 1] * u1 + Ef[3 * j + 2] * u2);
            }
        }
        // Gaussian elimination with partial pivoting
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int piv = c;
#pragma unroll
            for (int r = c + 1; r < 3; ++r)
                if (fabs(A[3 * r + c]) > fabs(A[3 * piv + c])) piv = r;
            if (piv != c) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const Real tmp = A[3 * c + j];
                    A[3 * c + j] = A[3 * piv + j];
                    A[3 * piv + j] = tmp;
                }
                const Real tb = b[c];
                b[c] = b[piv];
                b[piv] = tb;
            }
#pragma unroll
            for (int r = c + 1; r < 3; ++r) {
                const Real f = A[3 * r + c] / A[3 * c + c];
#pragma unroll
                for (int j = c; j < 3; ++j) A[3 * r + j] -= f * A[3 * c + j];
                b[r] -= f * b[c];
            }
        }
        Real x[3];
        x[2] = b[2] / A[8];
        x[1] = (b[1] - A[5] * x[2]) / A[4];
        x[0] = (b[0] - A[1] * x[1] - A[2] * x[2]) / A[0];
        Real *ps = psi + ((int64_t)a.task_slot[k] * G + g) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ps[i] = x[i];
            contrib[i] = (double)(wd * x[i]);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int wi = a.bwrite[3 * k + f];
            if (wi >= 0) {
                Real *o = bnd_out + ((int64_t)wi * G + g) * 3;
                o[0] = x[0];
                o[1] = x[1];
                o[2] = x[2];
            }
        }
    }
    // sum each run onto its first lane; every lane of the wavefront takes part in the
    // shuffles (idle lanes carry zeros, and a run never crosses a wavefront)
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
        Real *ra = reinterpret_cast<Real *>(a.run_acc) + ((a.k0 / TG + kg) * G + g) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) ra[i] = (Real)contrib[i];
    }
}

// Scalar-flux moments of every element: the sum of its runs' contributions, in a fixed
// order (run index), one thread per (element, group, moment).
template <typename Real>
__global__ void k_sn_gather(const Real *__restrict__ run_acc, const int *__restrict__ elem_off,
                            const int *__restrict__ elem_runs, double *__restrict__ phi_acc, int T, int G) {
    const int64_t n = (int64_t)T * G * 3;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int e = int(t / (3 * G));
        const int gi = int(t - (int64_t)e * 3 * G);
        double acc = 0.0;
        for (int j = elem_off[e]; j < elem_off[e + 1]; ++j) acc += (double)run_acc[(int64_t)elem_runs[j] * G * 3 + gi];
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
    if (precision == MOC_PREC_F64)
        k_sn_step<double><<<(unsigned)blocks, 256, 0, s>>>(a);
    else
        k_sn_step<float><<<(unsigned)blocks, 256, 0, s>>>(a);
    sn_check_launch();
}

void launch_sn_gather(const DevSN &d, hipStream_t s) {
    const int64_t n = (int64_t)d.T * d.G * 3;
    if (d.precision == MOC_PREC_F64)
        k_sn_gather<double><<<sn_grid(n), 256, 0, s>>>((const double *)d.run_acc, d.elem_off, d.elem_runs, d.phi_acc,
                                                        d.T, d.G);
    else
        k_sn_gather<float><<<sn_grid(n), 256, 0, s>>>((const float *)d.run_acc, d.elem_off, d.elem_runs, d.phi_acc,
                                                       d.T, d.G);
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
