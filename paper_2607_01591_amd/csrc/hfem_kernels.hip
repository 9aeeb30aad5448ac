// HIP kernels of libmoc's diffusion HFEM solver for gfx950 (CDNA4): the batched
// preassembly of every node's response matrices, the source update, the red-black
// response-matrix sweep, the flux reconstruction and the FP64 reductions of the power
// iteration (Sec. 2.1.2, Eq. HFEM_flux_response; Sec. 3.1).
//
// Per node and group, with the Legendre bases of hfem.h (volume u_i with
// (u_i, u_j) = V delta_ij, face v_m with <v_m, v_n>_f = A_f delta_mn):
//   A_ij  = D (grad u_i, grad u_j) + Sigma_r V delta_ij            (reaction matrix)
//   M_ri  = <v_m, u_i>_f = A_f t_ri,  r = (f, m)                    (face coupling)
//   C     = Lambda^-1 M A^-1,  Y = C M^T
//   J+    = R J- + B s,  R = (2I + Y)^-1 (Y - 2I) = I - 4 (2I + Y)^-1,  B = (2I + Y)^-1 C
//   phi   = A^-1 (s - M^T (J+ - J-))
// Since (2I + Y)^-1 = (I - R) / 4, the source term is B s = h - R h with h = C s / 4, the
// quarter of the face flux moments of A^-1 s; so each red-black update is the single
// product J+ = R (J- - h) + h and B is never formed. h costs one pass over A^-1 per
// outer iteration instead of one over B.
// The Legendre integrals are closed forms: on [-1, 1] with p_a = sqrt(2a+1) P_a,
// int p_a p_b = 2 delta_ab, int p_a' p_b' = sqrt((2a+1)(2b+1)) min(a,b) (min(a,b)+1) when
// a + b is even (else 0), and p_a(+-1) = sqrt(2a+1) (+-1)^a; so
// (d_x u_i, d_x u_j) = (2 V / hx^2) k(a_i, a_j) delta(b) delta(c), and the face factor
// t_ri = p_(a_d)(+-1) when the transverse degrees of u_i equal those of v_m, else 0
// (tabulated on the host).
#include <cmath>

#include "hfem_kernels.h"
#include "moc.h"
#include "moc_internal.h"

namespace moc {

__device__ __forceinline__ double hf_stiff1d(int a, int b) {
    if ((a + b) & 1) return 0.0;
    const int m = a < b ? a : b;
    return sqrt((double)((2 * a + 1) * (2 * b + 1))) * (double)(m * (m + 1));
}

__device__ __forceinline__ double hf_face_area(const double *h, int r, int Nfb) {
    const int d = (r / Nfb) >> 1;
    return d == 0 ? h[1] * h[2] : (d == 1 ? h[0] * h[2] : h[0] * h[1]);
}

// In-place Gauss-Jordan elimination with partial pivoting of the n x 2n augmented matrix
// W (row stride 2n, in LDS) by one wavefront: on return the right half holds the inverse
// of the left half. Lane r eliminates row r; the pivot row is chosen by lane 0.
__device__ void hf_gauss_jordan(double *W, int n, int *piv_sh, int *status) {
    const int lane = threadIdx.x;
    const int w = 2 * n;
    for (int c = 0; c < n; ++c) {
        if (lane == 0) {
            int piv = c;
            double best = fabs(W[c * w + c]);
            for (int r = c + 1; r < n; ++r) {
                const double v = fabs(W[r * w + c]);
                if (v > best) {
                    best = v;
                    piv = r;
                }
            }
            *piv_sh = piv;
            if (!(best > 0.0)) *status = 1;
        }
        __syncthreads();
        const int piv = *piv_sh;
        if (piv != c)
            for (int j = lane; j < w; j += 64) {
                const double t = W[c * w + j];
                W[c * w + j] = W[piv * w + j];
                W[piv * w + j] = t;
            }
        __syncthreads();
        const double inv = 1.0 / W[c * w + c];
        __syncthreads();
        for (int j = lane; j < w; j += 64) W[c * w + j] *= inv;
        __syncthreads();
        if (lane < n && lane != c) {
            const double f = W[lane * w + c];
            for (int j = 0; j < w; ++j) W[lane * w + j] -= f * W[c * w + j];
        }
        __syncthreads();
    }
}

// global block index and slot of a colour-sorted node-group (red blocks first)
__device__ __forceinline__ void hf_block_of(int64_t pg, int64_t red_pg, int npg_blk, int64_t nblk0, int64_t &blk,
                                           int &pl) {
    const int64_t lp = pg < red_pg ? pg : pg - red_pg;
    blk = lp / npg_blk + (pg < red_pg ? 0 : nblk0);
    pl = int(lp - (lp / npg_blk) * npg_blk);
}

// first node-group of a global block, and the end of its colour's range
__device__ __forceinline__ void hf_block_range(int64_t blk, int64_t red_pg, int64_t all_pg, int npg_blk, int64_t nblk0,
                                               int64_t &pg0, int64_t &pg_end) {
    if (blk < nblk0) {
        pg0 = blk * npg_blk;
        pg_end = red_pg;
    } else {
        pg0 = red_pg + (blk - nblk0) * npg_blk;
        pg_end = all_pg;
    }
}

struct HfAsmArgs {
    const int *perm, *mat, *vmode;
    const double *hdim, *diff, *sigr, *tface;
    void *R, *Ainv;   // double, or float when mat32
    int *status;
    int64_t red_pg, nblk0;
    int G, Np, Nfb, Nft, wsize, npg_blk, mat32;
};

// Preassembly: one wavefront per (colour-sorted node, group). Builds A and inverts it,
// forms C and 2I + Y and inverts that, and writes R and A^-1 in the blocked column layout
// of DevHF.
__global__ void __launch_bounds__(64) k_hf_assemble(HfAsmArgs a) {
    extern __shared__ double lds[];
    __shared__ int piv_sh;
    const int pg = blockIdx.x;
    const int G = a.G, Np = a.Np, Nfb = a.Nfb, Nft = a.Nft;
    const int p = pg / G, g = pg - p * G;
    const int lane = threadIdx.x;
    const int m = a.mat[a.perm[p]];
    const double h[3] = {a.hdim[3 * p], a.hdim[3 * p + 1], a.hdim[3 * p + 2]};
    const double V = h[0] * h[1] * h[2];
    const double D = a.diff[m * G + g], sr = a.sigr[m * G + g];
    double *W = lds;              // [n][2n] work
    double *Ai = W + a.wsize;     // [Np][Np] row-major
    double *Cm = Ai + Np * Np;    // [Nft][Np] row-major
    // reaction matrix | identity
    for (int idx = lane; idx < Np * Np; idx += 64) {
        const int i = idx / Np, j = idx - i * Np;
        const int *vi = a.vmode + 3 * i, *vj = a.vmode + 3 * j;
        double k = 0.0;
        if (vi[1] == vj[1] && vi[2] == vj[2]) k += hf_stiff1d(vi[0], vj[0]) / (h[0] * h[0]);
        if (vi[0] == vj[0] && vi[2] == vj[2]) k += hf_stiff1d(vi[1], vj[1]) / (h[1] * h[1]);
        if (vi[0] == vj[0] && vi[1] == vj[1]) k += hf_stiff1d(vi[2], vj[2]) / (h[2] * h[2]);
        W[i * 2 * Np + j] = D * 2.0 * V * k + (i == j ? sr * V : 0.0);
        W[i * 2 * Np + Np + j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    hf_gauss_jordan(W, Np, &piv_sh, a.status);
    for (int idx = lane; idx < Np * Np; idx += 64) {
        const int i = idx / Np, j = idx - i * Np;
        Ai[idx] = W[i * 2 * Np + Np + j];
    }
    __syncthreads();
    // C = Lambda^-1 M A^-1: C_rj = sum_i t_ri Ainv_ij
    for (int idx = lane; idx < Nft * Np; idx += 64) {
        const int r = idx / Np, j = idx - r * Np;
        double acc = 0.0;
        for (int i = 0; i < Np; ++i) {
            const double t = a.tface[r * Np + i];
            if (t != 0.0) acc += t * Ai[i * Np + j];
        }
        Cm[idx] = acc;
    }
    __syncthreads();
    // 2I + Y | identity, Y_rc = C_r . M_c = A_c sum_i C_ri t_ci
    for (int idx = lane; idx < Nft * Nft; idx += 64) {
        const int r = idx / Nft, c = idx - r * Nft;
        double acc = 0.0;
        for (int i = 0; i < Np; ++i) {
            const double t = a.tface[c * Np + i];
            if (t != 0.0) acc += Cm[r * Np + i] * t;
        }
        W[r * 2 * Nft + c] = hf_face_area(h, c, Nfb) * acc + (r == c ? 2.0 : 0.0);
        W[r * 2 * Nft + Nft + c] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    hf_gauss_jordan(W, Nft, &piv_sh, a.status);
    int64_t blk;
    int pl;
    hf_block_of(pg, a.red_pg, a.npg_blk, a.nblk0, blk, pl);
    const int nb = a.npg_blk;
    // R = I - 4 K^-1 (K = 2I + Y)
    for (int idx = lane; idx < Nft * Nft; idx += 64) {
        const int j = idx / Nft, i = idx - j * Nft;
        const double v = (i == j ? 1.0 : 0.0) - 4.0 * W[i * 2 * Nft + Nft + j];
        const int64_t o = ((blk * Nft + j) * nb + pl) * Nft + i;
        if (a.mat32)
            reinterpret_cast<float *>(a.R)[o] = (float)v;
        else
            reinterpret_cast<double *>(a.R)[o] = v;
    }
    // A^-1 (symmetric up to rounding; stored as computed)
    for (int idx = lane; idx < Np * Np; idx += 64) {
        const int k = idx / Np, i = idx - k * Np;
        const int64_t o = ((blk * Np + k) * nb + pl) * Np + i;
        if (a.mat32)
            reinterpret_cast<float *>(a.Ainv)[o] = (float)Ai[i * Np + k];
        else
            reinterpret_cast<double *>(a.Ainv)[o] = Ai[i * Np + k];
    }
}

// Per outer iteration, one block per global block of node-groups: the source moments
// s = V Q (from the previous flux, or V times a caller's emission moments), then
// a = A^-1 s, then h = C s / 4 = Lambda^-1 M a / 4 (face factor lists per face DoF).
// Emission: Q_g,i = chi_g F_i / k + sum_{g' != g} Sigma_s,g'->g phi_g',i (+ external).
template <int NP, int NFT, int KG, typename MT>
__global__ void __launch_bounds__(256) k_hf_prepare(const double *__restrict__ phi, const double *__restrict__ user,
                                                    const double *__restrict__ scal, const int *__restrict__ mat,
                                                    const int *__restrict__ perm, const double *__restrict__ vol,
                                                    const double *__restrict__ sigs, const double *__restrict__ nsf,
                                                    const double *__restrict__ chi, const double *__restrict__ qext,
                                                    const MT *__restrict__ Ainv, const int *__restrict__ rlist,
                                                    const double *__restrict__ rval, double *__restrict__ s,
                                                    double *__restrict__ h, int64_t red_pg, int64_t all_pg,
                                                    int64_t nblk0, int G_, int Np_, int Nft_, int nr) {
    // NP moments, and KG groups and NFT face DoFs when non-zero, known at compile time, so
    // the loops over groups and moments unroll and their loads issue together
    const int G = KG > 0 ? KG : G_;
    const int Nft = NFT > 0 ? NFT : Nft_;
    constexpr int Np = NP;
    (void)Np_;
    extern __shared__ double sh[];
    const int npg_blk = 256 / Nft;
    double *sv = sh;                    // [npg_blk][Np]
    double *av = sh + npg_blk * Np;     // [npg_blk][Np]
    const int64_t blk = blockIdx.x;
    int64_t pg0, pg_end;
    hf_block_range(blk, red_pg, all_pg, npg_blk, nblk0, pg0, pg_end);
    const double inv_k = 1.0 / scal[kHfK];
    for (int t = threadIdx.x; t < npg_blk * Np; t += blockDim.x) {
        const int pl = t / Np, k = t - pl * Np;
        const int64_t pg = pg0 + pl;
        if (pg >= pg_end) continue;
        const int p = int(pg / G), g = int(pg - (int64_t)p * G);
        const int e = perm[p];
        const int64_t src = ((int64_t)e * G + g) * Np + k;
        double q;
        if (user) {
            q = user[src];
        } else {
            const int m = mat[e];
            const double *ph = phi + (int64_t)e * G * Np + k;
            const double cg = chi[m * G + g] * inv_k;
            const double *sg = sigs + (int64_t)m * G * G + g;
            q = qext ? qext[src] : 0.0;
#pragma unroll
            for (int gp = 0; gp < G; ++gp) q += (cg * nsf[m * G + gp] + (gp != g ? sg[gp * G] : 0.0)) * ph[gp * Np];
        }
        const double v = vol[e] * q;
        sv[t] = v;
        s[pg * Np + k] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < npg_blk * Np; t += blockDim.x) {
        const int pl = t / Np, i = t - pl * Np;
        if (pg0 + pl >= pg_end) continue;
        const MT *Ab = Ainv + blk * Np * npg_blk * Np + t;
        const double *x = sv + pl * Np;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < Np; ++k) acc += (double)Ab[(int64_t)k * npg_blk * Np] * x[k];
        av[t] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < npg_blk * Nft; t += blockDim.x) {
        const int pl = t / Nft, r = t - pl * Nft;
        const int64_t pg = pg0 + pl;
        if (pg >= pg_end) continue;
        double acc = 0.0;
        for (int q = 0; q < nr; ++q) {
            const int k = rlist[r * nr + q];
            if (k < 0) break;
            acc += rval[r * nr + q] * av[pl * Np + k];
        }
        h[pg * Nft + r] = 0.25 * acc;
    }
}

// Outgoing partial currents are stored face-major, [colour-sorted node][face][group][mode]:
// the G groups of one face of a node are one contiguous run, so the neighbours of a block
// (which holds consecutive groups of the same nodes) read whole cache lines.
__device__ __forceinline__ int64_t hf_jp_index(int p, int f, int g, int mm, int G, int Nfb) {
    return (((int64_t)p * 6 + f) * G + g) * Nfb + mm;
}

// Incoming partial current of face DoF i of colour-sorted node p, group g.
__device__ __forceinline__ double hf_incoming(const double *__restrict__ jp, const int *__restrict__ nbr, int p, int g,
                                              int i, int G, int Nfb) {
    const int f = i / Nfb, mm = i - f * Nfb;
    const int code = nbr[6 * p + f];
    if (code >= 0) return jp[hf_jp_index(code, f ^ 1, g, mm, G, Nfb)];
    if (code == kHfReflect) return jp[hf_jp_index(p, f, g, mm, G, Nfb)];
    return 0.0;
}

// Red-black half sweep over the blocks [blk0, blk0 + gridDim.x) of one colour
// (Eq. HFEM_flux_response): J+ = R J- + B s = R (J- - h) + h. Thread (slot, i) holds
// row i of its node-group: it loads that row of R (each column of the block is one
// contiguous run) while J- - h of the block's node-groups is gathered into LDS (a node's
// own outgoing currents feed its reflective faces, so they are read before any is
// overwritten), then forms the product.
template <int NFT, typename MT>
__global__ void __launch_bounds__(256) k_hf_rb(const MT *__restrict__ R, const double *__restrict__ h,
                                               double *__restrict__ jp, const int *__restrict__ nbr, int64_t blk0,
                                               int64_t red_pg, int64_t all_pg, int64_t nblk0, int G, int Nfb) {
    constexpr int NPG = 256 / NFT;
    __shared__ double jm[256];
    const int64_t blk = blk0 + blockIdx.x;
    int64_t pg0, pg_end;
    hf_block_range(blk, red_pg, all_pg, NPG, nblk0, pg0, pg_end);
    const int t = threadIdx.x;
    const int pl = t / NFT, i = t - pl * NFT;
    const int64_t pg = pg0 + pl;
    const bool active = pl < NPG && pg < pg_end;
    double row[NFT];
    double acc = 0.0;
    int p = 0, g = 0;
    if (active) {
        const MT *Rb = R + blk * NFT * NPG * NFT + t;
#pragma unroll
        for (int j = 0; j < NFT; ++j) row[j] = (double)Rb[j * NPG * NFT];
        acc = h[pg * NFT + i];
        p = int(pg / G);
        g = int(pg - (int64_t)p * G);
        jm[t] = hf_incoming(jp, nbr, p, g, i, G, Nfb) - acc;
    }
    __syncthreads();
    if (active) {
        const double *x = jm + pl * NFT;
#pragma unroll
        for (int j = 0; j < NFT; ++j) acc += row[j] * x[j];
        const int f = i / Nfb;
        jp[hf_jp_index(p, f, g, i - f * Nfb, G, Nfb)] = acc;
    }
}

// phi = A^-1 (s - M^T (J+ - J-)), written in node order, one block per global block of
// node-groups. Thread (slot, i) loads row i of A^-1 for its node-group while the net
// currents are gathered into LDS; then u = s - M^T j (M = face area x face factor, from
// the compact per-moment lists of non-zero face factors), then phi_i = sum_k Ainv_ik u_k.
template <int NP, int NFT, int KG, typename MT>
__global__ void __launch_bounds__(256) k_hf_reconstruct(const MT *__restrict__ Ainv, const int *__restrict__ flist,
                                                        const double *__restrict__ fval, const double *__restrict__ hdim,
                                                        const double *__restrict__ s, const double *__restrict__ jp,
                                                        const int *__restrict__ nbr, const int *__restrict__ perm,
                                                        double *__restrict__ phi, int64_t red_pg, int64_t all_pg,
                                                        int64_t nblk0, int G_, int Nfb_, int Nft_) {
    // face DoFs (NFT) and groups (KG) known at compile time when non-zero: the divisions and
    // index products of the gathers fold
    const int G = KG > 0 ? KG : G_;
    const int Nft = NFT > 0 ? NFT : Nft_, Nfb = NFT > 0 ? NFT / 6 : Nfb_;
    extern __shared__ double sh[];
    const int npg_blk = 256 / Nft;
    double *net = sh;                   // [npg_blk][Nft]
    double *u = sh + npg_blk * Nft;     // [npg_blk][NP]
    const int64_t blk = blockIdx.x;
    int64_t pg0, pg_end;
    hf_block_range(blk, red_pg, all_pg, npg_blk, nblk0, pg0, pg_end);
    for (int t = threadIdx.x; t < npg_blk * Nft; t += blockDim.x) {
        const int pl = t / Nft, i = t - pl * Nft;
        const int64_t pg = pg0 + pl;
        if (pg < pg_end) {
            const int p = int(pg / G), g = int(pg - (int64_t)p * G);
            const int f = i / Nfb;
            net[t] = jp[hf_jp_index(p, f, g, i - f * Nfb, G, Nfb)] - hf_incoming(jp, nbr, p, g, i, G, Nfb);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < npg_blk * NP; t += blockDim.x) {
        const int pl = t / NP, k = t - pl * NP;
        const int64_t pg = pg0 + pl;
        if (pg >= pg_end) continue;
        const int p = int(pg / G);
        const double hx = hdim[3 * p], hy = hdim[3 * p + 1], hz = hdim[3 * p + 2];
        const double area[3] = {hy * hz, hx * hz, hx * hy};
        double w = 0.0;
        for (int q = 0; q < 6; ++q) {
            const int c = flist[k * 6 + q];
            if (c < 0) break;
            w += area[(c / Nfb) >> 1] * fval[k * 6 + q] * net[pl * Nft + c];
        }
        u[t] = s[pg * NP + k] - w;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < npg_blk * NP; t += blockDim.x) {
        const int pl = t / NP, i = t - pl * NP;
        const int64_t pg = pg0 + pl;
        if (pg >= pg_end) continue;
        const int p = int(pg / G), g = int(pg - (int64_t)p * G);
        const MT *Ab = Ainv + blk * NP * npg_blk * NP + t;
        const double *uv = u + pl * NP;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) acc += (double)Ab[k * npg_blk * NP] * uv[k];
        phi[((int64_t)perm[p] * G + g) * NP + i] = acc;
    }
}

__device__ __forceinline__ double hf_block_sum(double v, double *sh) {
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

// partials of sum_e V nuSigma_f phi_0 for the new and the old iterate
__global__ void k_hf_fission(const double *__restrict__ phi_new, const double *__restrict__ phi_old,
                             const double *__restrict__ vol, const int *__restrict__ mat, const double *__restrict__ nsf,
                             double *__restrict__ partials, int N, int G, int Np) {
    __shared__ double sh[16];
    double fn = 0.0, fo = 0.0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
        const int m = mat[e];
        double xn = 0.0, xo = 0.0;
        for (int g = 0; g < G; ++g) {
            xn += nsf[m * G + g] * phi_new[((int64_t)e * G + g) * Np];
            xo += nsf[m * G + g] * phi_old[((int64_t)e * G + g) * Np];
        }
        fn += vol[e] * xn;
        fo += vol[e] * xo;
    }
    fn = hf_block_sum(fn, sh);
    fo = hf_block_sum(fo, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = fn;
        partials[2 * blockIdx.x + 1] = fo;
    }
}

// Single block: k <- k F_new / F_old (eigen) or k kept (fixed source).
__global__ void k_hf_eigen(const double *__restrict__ partials, int nblk, double *__restrict__ scal, int fixed_source) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    a = hf_block_sum(a, sh);
    b = hf_block_sum(b, sh);
    if (threadIdx.x == 0) {
        const double k = scal[kHfK];
        scal[kHfKPrev] = k;
        scal[kHfFnew] = a;
        scal[kHfFold] = b;
        if (!fixed_source) {
            scal[kHfK] = k * a / b;
            scal[kHfDk] = fabs(scal[kHfK] - k);
        } else {
            scal[kHfDk] = 0.0;
        }
    }
}

// partials of the residual norms: eigen, the normalised fission-rate shapes
// a = nuSigma_f phi_0 / F_new, b = ... / F_old: sum V (a - b)^2, sum V a^2; fixed source:
// sum over nodes and groups of V (phi_0,new - phi_0,old)^2 and V phi_0,new^2.
__global__ void k_hf_residual_partials(const double *__restrict__ phi_new, const double *__restrict__ phi_old,
                                       const double *__restrict__ vol, const int *__restrict__ mat,
                                       const double *__restrict__ nsf, const double *__restrict__ scal,
                                       double *__restrict__ partials, int N, int G, int Np, int fixed_source) {
    __shared__ double sh[16];
    const double rn = fixed_source ? 1.0 : 1.0 / scal[kHfFnew];
    const double ro = fixed_source ? 1.0 : 1.0 / scal[kHfFold];
    double num = 0.0, den = 0.0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
        const int m = mat[e];
        if (fixed_source) {
            for (int g = 0; g < G; ++g) {
                const double a = phi_new[((int64_t)e * G + g) * Np], b = phi_old[((int64_t)e * G + g) * Np];
                num += vol[e] * (a - b) * (a - b);
                den += vol[e] * a * a;
            }
        } else {
            double xn = 0.0, xo = 0.0;
            for (int g = 0; g < G; ++g) {
                xn += nsf[m * G + g] * phi_new[((int64_t)e * G + g) * Np];
                xo += nsf[m * G + g] * phi_old[((int64_t)e * G + g) * Np];
            }
            const double a = xn * rn, b = xo * ro;
            num += vol[e] * (a - b) * (a - b);
            den += vol[e] * a * a;
        }
    }
    num = hf_block_sum(num, sh);
    den = hf_block_sum(den, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = num;
        partials[2 * blockIdx.x + 1] = den;
    }
}

__global__ void k_hf_residual_final(const double *__restrict__ partials, int nblk, double *__restrict__ scal) {
    __shared__ double sh[16];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    a = hf_block_sum(a, sh);
    b = hf_block_sum(b, sh);
    if (threadIdx.x == 0) scal[kHfRes] = sqrt(a / (b > 1e-300 ? b : 1e-300));
}

// outgoing currents to node order, [node][group][face DoF]
__global__ void k_hf_currents_to_nodes(const double *__restrict__ jp, const int *__restrict__ perm,
                                       double *__restrict__ out, int N, int G, int Nfb) {
    const int Nft = 6 * Nfb;
    const int64_t n = (int64_t)N * G * Nft;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pg = t / Nft;
        const int i = int(t - pg * Nft);
        const int p = int(pg / G), g = int(pg - (int64_t)p * G);
        const int f = i / Nfb;
        out[((int64_t)perm[p] * G + g) * Nft + i] = jp[hf_jp_index(p, f, g, i - f * Nfb, G, Nfb)];
    }
}

// cold flux: phi_0 = 1, higher moments 0
__global__ void k_hf_cold(double *__restrict__ phi, int64_t n, int Np) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        phi[t] = (t % Np) == 0 ? 1.0 : 0.0;
}

__global__ void k_hf_fill(double *__restrict__ p, int64_t n, double v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

// ----------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------

static void hf_check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(MOC_EHIP, hipGetErrorString(e));
}

static int hf_grid(int64_t n, int block = 256, int cap = 16384) {
    const int64_t b = (n + block - 1) / block;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

void launch_hf_assemble(const DevHF &d, hipStream_t s) {
    HfAsmArgs a{};
    a.perm = d.perm;
    a.mat = d.mat;
    a.vmode = d.vmode;
    a.tface = d.tface;
    a.hdim = d.hdim;
    a.diff = d.diff;
    a.sigr = d.sigr;
    a.R = d.R;
    a.Ainv = d.Ainv;
    a.mat32 = d.mat32;
    a.status = d.status;
    a.red_pg = (int64_t)d.n_red * d.G;
    a.nblk0 = d.nblk[0];
    a.npg_blk = d.npg_blk;
    a.G = d.G;
    a.Np = d.Np;
    a.Nfb = d.Nfb;
    a.Nft = d.Nft;
    a.wsize = 2 * (d.Np > d.Nft ? d.Np * d.Np : d.Nft * d.Nft);
    const size_t lds = sizeof(double) * ((size_t)a.wsize + (size_t)d.Np * d.Np + (size_t)d.Nft * d.Np);
    const int64_t npg = (int64_t)d.N * d.G;
    if (npg <= 0) return;
    k_hf_assemble<<<(unsigned)npg, 64, lds, s>>>(a);
    hf_check_launch();
}

template <int NP, int NFT, int KG, typename MT>
static void hf_prepare_t(const DevHF &d, const double *phi, const double *user, int64_t nb, size_t lds, hipStream_t s) {
    k_hf_prepare<NP, NFT, KG, MT><<<(unsigned)nb, 256, lds, s>>>(phi, user, d.scal, d.mat, d.perm, d.vol, d.sigs, d.nsf, d.chi, d.qext,
                                                    (const MT *)d.Ainv, d.rlist, d.rval, d.s, d.bq,
                                                    (int64_t)d.n_red * d.G, (int64_t)d.N * d.G, d.nblk[0], d.G, d.Np,
                                                    d.Nft, d.nr);
}

// the 7-group shapes with the group count (and for face order 1 the face DoFs) known at
// compile time, other counts general
template <int NP>
static void hf_prepare_np(const DevHF &d, const double *phi, const double *user, int64_t nb, size_t lds, hipStream_t s) {
    if (NP == 10 && d.G == 7 && d.Nft == 18) {   // volume order 2, face order 1, 7 groups
        if (d.mat32) hf_prepare_t<NP, 18, 7, float>(d, phi, user, nb, lds, s);
        else hf_prepare_t<NP, 18, 7, double>(d, phi, user, nb, lds, s);
    } else if (d.G == 7) {
        if (d.mat32) hf_prepare_t<NP, 0, 7, float>(d, phi, user, nb, lds, s);
        else hf_prepare_t<NP, 0, 7, double>(d, phi, user, nb, lds, s);
    } else {
        if (d.mat32) hf_prepare_t<NP, 0, 0, float>(d, phi, user, nb, lds, s);
        else hf_prepare_t<NP, 0, 0, double>(d, phi, user, nb, lds, s);
    }
}

void launch_hf_prepare(const DevHF &d, const double *phi, const double *user, hipStream_t s) {
    const int64_t nb = d.nblk[0] + d.nblk[1];
    if (nb <= 0) return;
    const size_t lds = sizeof(double) * (size_t)d.npg_blk * 2 * d.Np;
    switch (d.Np) {
    case 1: hf_prepare_np<1>(d, phi, user, nb, lds, s); break;
    case 4: hf_prepare_np<4>(d, phi, user, nb, lds, s); break;
    case 10: hf_prepare_np<10>(d, phi, user, nb, lds, s); break;
    case 20: hf_prepare_np<20>(d, phi, user, nb, lds, s); break;
    case 35: hf_prepare_np<35>(d, phi, user, nb, lds, s); break;
    default: throw Error(MOC_EINVAL, "hfem: unsupported number of moments");
    }
    hf_check_launch();
}

template <int NFT, typename MT>
static void hf_rb_t(const DevHF &d, int64_t nb, int64_t blk0, hipStream_t s) {
    k_hf_rb<NFT, MT><<<(unsigned)nb, 256, 0, s>>>((const MT *)d.R, d.bq, d.jp, d.nbr, blk0, (int64_t)d.n_red * d.G,
                                                  (int64_t)d.N * d.G, d.nblk[0], d.G, d.Nfb);
}

void launch_hf_rb(const DevHF &d, int colour, hipStream_t s) {
    const int64_t nb = d.nblk[colour];
    if (nb <= 0) return;
    const int64_t blk0 = colour == 0 ? 0 : d.nblk[0];
    switch (d.Nft * 2 + (d.mat32 ? 1 : 0)) {
    case 12: hf_rb_t<6, double>(d, nb, blk0, s); break;
    case 13: hf_rb_t<6, float>(d, nb, blk0, s); break;
    case 36: hf_rb_t<18, double>(d, nb, blk0, s); break;
    case 37: hf_rb_t<18, float>(d, nb, blk0, s); break;
    case 72: hf_rb_t<36, double>(d, nb, blk0, s); break;
    case 73: hf_rb_t<36, float>(d, nb, blk0, s); break;
    default: throw Error(MOC_EINVAL, "hfem: unsupported number of face DoFs");
    }
    hf_check_launch();
}

template <int NP, int NFT, int KG, typename MT>
static void hf_reconstruct_t(const DevHF &d, double *phi_out, int64_t nb, size_t lds, hipStream_t s) {
    k_hf_reconstruct<NP, NFT, KG, MT><<<(unsigned)nb, 256, lds, s>>>((const MT *)d.Ainv, d.flist, d.fval, d.hdim, d.s, d.jp, d.nbr,
                                                            d.perm, phi_out, (int64_t)d.n_red * d.G, (int64_t)d.N * d.G,
                                                            d.nblk[0], d.G, d.Nfb, d.Nft);
}

template <int NP> static void hf_reconstruct_np(const DevHF &d, double *phi_out, int64_t nb, size_t lds, hipStream_t s) {
    if (d.mat32)
        hf_reconstruct_t<NP, 0, 0, float>(d, phi_out, nb, lds, s);
    else
        hf_reconstruct_t<NP, 0, 0, double>(d, phi_out, nb, lds, s);
}

void launch_hf_reconstruct(const DevHF &d, double *phi_out, hipStream_t s) {
    const int64_t nb = d.nblk[0] + d.nblk[1];
    if (nb <= 0) return;
    const size_t lds = sizeof(double) * (size_t)d.npg_blk * (d.Nft + d.Np);
    if (d.Np == 10 && d.Nft == 18 && d.G == 7) {   // volume order 2, face order 1, 7 groups
        if (d.mat32) hf_reconstruct_t<10, 18, 7, float>(d, phi_out, nb, lds, s);
        else hf_reconstruct_t<10, 18, 7, double>(d, phi_out, nb, lds, s);
        hf_check_launch();
        return;
    }
    switch (d.Np) {
    case 1: hf_reconstruct_np<1>(d, phi_out, nb, lds, s); break;
    case 4: hf_reconstruct_np<4>(d, phi_out, nb, lds, s); break;
    case 10: hf_reconstruct_np<10>(d, phi_out, nb, lds, s); break;
    case 20: hf_reconstruct_np<20>(d, phi_out, nb, lds, s); break;
    case 35: hf_reconstruct_np<35>(d, phi_out, nb, lds, s); break;
    default: throw Error(MOC_EINVAL, "hfem: unsupported number of moments");
    }
    hf_check_launch();
}

void launch_hf_fission(const DevHF &d, const double *phi_new, const double *phi_old, hipStream_t s) {
    k_hf_fission<<<kHfReduceBlocks, 256, 0, s>>>(phi_new, phi_old, d.vol, d.mat, d.nsf, d.partials, d.N, d.G, d.Np);
    hf_check_launch();
}

void launch_hf_eigen(const DevHF &d, int fixed_source, hipStream_t s) {
    k_hf_eigen<<<1, 256, 0, s>>>(d.partials, kHfReduceBlocks, d.scal, fixed_source);
    hf_check_launch();
}

void launch_hf_residual(const DevHF &d, const double *phi_new, const double *phi_old, int fixed_source,
                        hipStream_t s) {
    k_hf_residual_partials<<<kHfReduceBlocks, 256, 0, s>>>(phi_new, phi_old, d.vol, d.mat, d.nsf, d.scal, d.partials,
                                                           d.N, d.G, d.Np, fixed_source);
    k_hf_residual_final<<<1, 256, 0, s>>>(d.partials, kHfReduceBlocks, d.scal);
    hf_check_launch();
}

void launch_hf_currents_to_nodes(const DevHF &d, double *out, hipStream_t s) {
    k_hf_currents_to_nodes<<<hf_grid((int64_t)d.N * d.G * d.Nft), 256, 0, s>>>(d.jp, d.perm, out, d.N, d.G, d.Nfb);
    hf_check_launch();
}

void launch_hf_cold(const DevHF &d, double *phi, hipStream_t s) {
    const int64_t n = (int64_t)d.N * d.G * d.Np;
    k_hf_cold<<<hf_grid(n), 256, 0, s>>>(phi, n, d.Np);
    hf_check_launch();
}

void launch_hf_fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    k_hf_fill<<<hf_grid(n), 256, 0, s>>>(p, n, v);
    hf_check_launch();
}

}  // namespace moc
