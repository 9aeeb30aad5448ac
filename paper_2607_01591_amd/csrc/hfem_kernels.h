// Device state and kernel launchers of the diffusion HFEM solver (see hfem_kernels.hip).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace moc {

// neighbour codes per (colour-sorted node, face)
constexpr int kHfReflect = -1;   // reflective side: J- = own J+ on that face
constexpr int kHfVacuum = -2;    // vacuum side: J- = 0
// >= 0: colour-sorted position of the neighbour across the face

constexpr int kHfMaxMoments = 35;   // volume order 4 in 3D
constexpr int kHfMaxFaceDofs = 36;  // face order 2: 6 modes on each of 6 faces

struct DevHF {
    int N = 0, G = 0, M = 0, Np = 0, Nfb = 0, Nft = 0, n_red = 0;
    int *perm = nullptr;     // [N] colour-sorted position -> node
    int *pos = nullptr;      // [N] node -> colour-sorted position
    int *nbr = nullptr;      // [N][6] by colour-sorted position
    double *hdim = nullptr;  // [N][3] by colour-sorted position
    int *mat = nullptr;      // [N] by node
    double *vol = nullptr;   // [N] by node
    double *diff = nullptr, *sigr = nullptr;   // [M][G]
    double *sigs = nullptr;  // [M][G][G] from -> to
    double *nsf = nullptr, *chi = nullptr;     // [M][G]
    int *vmode = nullptr;    // [Np][3] Legendre degrees of the volume modes
    // Node-groups (colour-sorted node, group) are dealt to blocks of npg_blk, colour by
    // colour (the red blocks first; the last block of a colour may be partial). Within a
    // block each matrix is stored column by column with the block's node-groups
    // interleaved: entry (row i, column j) of slot pl sits at
    //   [block][j][pl][i]
    // so that one column of every node-group of a block is one contiguous run.
    int npg_blk = 0;         // node-groups per block (256 / Nft)
    int64_t nblk[2] = {0, 0};
    int mat32 = 0;           // R and A^-1 stored in FP32 (products still accumulate in FP64)
    void *R = nullptr;       // [blocks][Nft][npg_blk][Nft]
    void *Ainv = nullptr;    // [blocks][Np][npg_blk][Np]
    double *tface = nullptr; // [Nft][Np] face factors t (M = face area x t)
    int *flist = nullptr;    // [Np][6] face DoFs with t != 0 for each moment (-1 ends the list)
    double *fval = nullptr;  // [Np][6] their face factors
    int nr = 0;              // length of the per-face-DoF lists
    int *rlist = nullptr;    // [Nft][nr] moments with t != 0 for each face DoF (-1 ends the list)
    double *rval = nullptr;  // [Nft][nr] their face factors
    double *jp = nullptr;    // [N][6][G][Nfb] outgoing partial currents, colour-sorted, face-major
    double *s = nullptr;     // [N][G][Np] source moments (u_i, Q), colour-sorted
    double *bq = nullptr;    // [N][G][Nft] h = C s / 4 (B s = h - R h)
    double *phi[2] = {nullptr, nullptr};   // [N][G][Np] by node
    double *qext = nullptr;  // [N][G][Np] by node
    double *partials = nullptr, *scal = nullptr;
    int *status = nullptr;   // preassembly flags (non-zero: a singular pivot)
};

// indices into DevHF::scal
enum { kHfK = 0, kHfKPrev = 1, kHfFnew = 2, kHfFold = 3, kHfRes = 4, kHfDk = 5, kHfCount = 8 };
constexpr int kHfReduceBlocks = 256;

void launch_hf_assemble(const DevHF &d, hipStream_t s);
// s, A^-1 s and h from the previous flux phi (user == nullptr) or a caller's emission moments
void launch_hf_prepare(const DevHF &d, const double *phi, const double *user, hipStream_t s);
void launch_hf_rb(const DevHF &d, int colour, hipStream_t s);
void launch_hf_reconstruct(const DevHF &d, double *phi_out, hipStream_t s);
void launch_hf_fission(const DevHF &d, const double *phi_new, const double *phi_old, hipStream_t s);
void launch_hf_eigen(const DevHF &d, int fixed_source, hipStream_t s);
void launch_hf_residual(const DevHF &d, const double *phi_new, const double *phi_old, int fixed_source, hipStream_t s);
void launch_hf_currents_to_nodes(const DevHF &d, double *out, hipStream_t s);
void launch_hf_cold(const DevHF &d, double *phi, hipStream_t s);
void launch_hf_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace moc
