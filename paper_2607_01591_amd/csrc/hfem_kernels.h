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
    int *fmode = nullptr;    // [Nfb][2] degrees of the face modes
    // per (colour-sorted node, group), each column-major: column index outer, row inner
    double *R = nullptr;     // [N][G][Nft cols][Nft rows]
    double *B = nullptr;     // [N][G][Np cols][Nft rows]
    double *Ainv = nullptr;  // [N][G][Np cols][Np rows]
    double *P = nullptr;     // [N][G][Nft cols][Np rows]  (A^-1 M^T)
    double *jp = nullptr;    // [N][G][Nft] outgoing partial currents, colour-sorted
    double *s = nullptr;     // [N][G][Np] source moments (u_i, Q), colour-sorted
    double *bq = nullptr;    // [N][G][Nft] B s
    double *phi[2] = {nullptr, nullptr};   // [N][G][Np] by node
    double *qext = nullptr;  // [N][G][Np] by node
    double *partials = nullptr, *scal = nullptr;
    int *status = nullptr;   // preassembly flags (non-zero: a singular pivot)
};

// indices into DevHF::scal
enum { kHfK = 0, kHfKPrev = 1, kHfFnew = 2, kHfFold = 3, kHfRes = 4, kHfDk = 5, kHfCount = 8 };
constexpr int kHfReduceBlocks = 256;

void launch_hf_assemble(const DevHF &d, hipStream_t s);
void launch_hf_source(const DevHF &d, const double *phi, hipStream_t s);
void launch_hf_user_source(const DevHF &d, const double *src, hipStream_t s);
void launch_hf_bq(const DevHF &d, hipStream_t s);
void launch_hf_rb(const DevHF &d, int colour, hipStream_t s);
void launch_hf_reconstruct(const DevHF &d, double *phi_out, hipStream_t s);
void launch_hf_fission(const DevHF &d, const double *phi_new, const double *phi_old, hipStream_t s);
void launch_hf_eigen(const DevHF &d, int fixed_source, hipStream_t s);
void launch_hf_residual(const DevHF &d, const double *phi_new, const double *phi_old, int fixed_source, hipStream_t s);
void launch_hf_currents_to_nodes(const DevHF &d, double *out, hipStream_t s);
void launch_hf_cold(const DevHF &d, double *phi, hipStream_t s);
void launch_hf_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace moc
