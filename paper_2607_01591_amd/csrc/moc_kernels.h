// Device-side state and kernel launchers of libmoc (see moc_kernels.hip for layouts).
#pragma once

#include "moc_internal.h"

namespace moc {

// indices into the device scalar array
enum { kScalK = 0, kScalKPrev = 1, kScalF = 2, kScalRes = 3, kScalDk = 4, kScalFsum = 5, kScalCount = 8 };

// table of (1 - e^-x)/x for the FP32 table exponential: kExpTableN points on [0, kExpTableMax]
constexpr int kExpTableN = 2048;
constexpr float kExpTableMax = 16.0f;

// largest tally window the sweep kernel accepts (slots per window)
constexpr int kMaxSlots = 256;

// fixed number of blocks for the FP64 reductions (partials are summed in block order)
constexpr int kReduceBlocks = 512;

struct SweepArgs {
    const void *segs;             // SegF / SegD, per window [step][64 lanes]
    const int64_t *batch_win;     // [nb + 1] window range of each batch
    const int64_t *win_entry_off; // [nw] first entry of each window
    const int *win_nsteps;        // [nw]
    const int64_t *win_tab_off;   // [nw] first slot-table entry of each window
    const int *win_nslots;        // [nw]
    const int *win_tab;           // slot -> internal region
    int cap;                      // LDS tally rows per group (>= every window's slot count)
    const int *batch_angle;       // [nb]
    const int *batch_of_block;    // [nb] batch swept by workgroup column blockIdx.x
    const void *xsq;           // Real [R][Gp][2] (Sigma_t, qhat)
    const void *psi_in;        // Real [2][P][Gp][nslots]
    void *psi_out;
    const int *link;           // [2][nslots] -> sense' * nslots + slot', or -1
    const unsigned char *fed;  // [2][nslots] 1 if some link feeds this incoming slot
    const void *coef;          // Real [NA][P]
    const void *inv_sin;       // Real [P]
    const float *exp_table;    // [ExpTable::kN] (FP32 table mode)
    double *tally;             // [R][Gp]
    const unsigned *tally_bound; // [Gp] FP32 sweep: max(|qhat|, |psi_in|) per group (float bits)
    double *exit_canon;        // optional [T][2][P][G]
    const int *canon_of_slot;  // [nslots] canonical track or -1
    int nslots, Gp, G;
    int n_real;                // regions; tally rows at and above it are coarse surfaces
};

struct DevProblem {
    int R = 0, G = 0, Gp = 0, M = 0, P = 0, NA = 0, T = 0;
    int nb = 0, nslots = 0, gb = 1, n_gb = 1;
    int precision = MOC_PREC_F32, exp_mode = MOC_EXP_POLY;
    // per material, FP64
    double *sigt_m = nullptr, *sigs_m = nullptr, *nsf_m = nullptr, *chi_m = nullptr;
    // per internal region
    int *mat = nullptr, *user_of = nullptr;
    double *V = nullptr;
    void *xsq = nullptr;   // Real [R][Gp][2] (Sigma_t, qhat)
    double *tally = nullptr;
    double *phi[2] = {nullptr, nullptr};
    double *qext = nullptr;
    // tracks and tally windows
    void *segs = nullptr;
    int64_t *batch_win = nullptr, *win_entry_off = nullptr, *win_tab_off = nullptr;
    int *win_nsteps = nullptr, *win_nslots = nullptr, *win_tab = nullptr;
    int *batch_angle = nullptr;
    int *batch_of_block = nullptr;   // [nb] see make_batch_order
    int cap = 256, max_slots = 1;
    void *psi[2] = {nullptr, nullptr};
    int *link = nullptr;
    unsigned char *fed = nullptr;
    int *entry_region = nullptr;   // [2][nslots] internal region entered first, -1 dummy
    int *slot_of_canon = nullptr, *canon_of_slot = nullptr;
    void *coef = nullptr, *inv_sin = nullptr;
    float *exp_table = nullptr;
    // reductions
    double *partials = nullptr, *scal = nullptr;
    unsigned *tally_bound = nullptr;   // [Gp] see SweepArgs
};

// Coarse mesh (CMFD) device state; see moc_cmfd.hip.
// exchange area of the cooperative coarse solve: two 128-byte lines per block (at most
// 256 blocks) and one line for the abort word
constexpr int64_t kCmfdRedDoubles = (int64_t)256 * 2 * 16 + 16;
constexpr int kCmfdVectors = 11;   // solver vectors of the coarse solve

struct DevCoarse {
    int C = 0, Ns = 0, nadj = 0;
    int *cell_of = nullptr;           // [R] internal region -> cell
    int64_t *cell_reg_off = nullptr;  // [C + 1] internal regions of each cell
    int *cell_reg = nullptr;          // [R]
    int *entry_cell = nullptr;        // [2][nslots] cell of the first region per incoming track-sense, -1
    int64_t *adj_off = nullptr;       // [C + 1] surfaces of each cell
    int *adj_surf = nullptr, *adj_nbr = nullptr;  // [nadj] surface id, neighbour cell (-1 = boundary)
    double *adj_sign = nullptr;       // [nadj] +1 if the surface's positive orientation leaves the cell
    double *adj_L = nullptr, *adj_h = nullptr, *adj_hn = nullptr;  // [nadj] shared length, centroid distances
    double *hsum = nullptr;           // [C][2 + 4 G + G^2] homogenisation sums
    double *Bs = nullptr, *Binv = nullptr;  // [C][G][G] diagonal blocks and their inverses
    double *Aoff = nullptr;           // [nadj][G] neighbour couplings
    double *phih = nullptr, *Dc = nullptr, *Ldiag = nullptr, *fchi = nullptr, *fnsf = nullptr;  // [C][G]
    double *vec = nullptr;            // [kCmfdVectors][C G] solver vectors
    double *ratio = nullptr;          // [C][G]
    double *stats = nullptr;          // [4] outer, inner iterations, coarse k
    int *piv = nullptr;               // [C][G]
    double *red = nullptr;            // [kCmfdRedDoubles] block exchange lines of the cooperative solve
    bool grid_ok = false;             // the device supports cooperative launches
    int blocks = 0;                   // coarse solve blocks (0 automatic, 1 one workgroup)
    double tol = 1e-5, shift = 0.02;
    int max_outer = 20, max_inner = 200;
    int max_deg = 0;                  // most surfaces of any cell
};

void launch_cmfd(const DevProblem &d, const DevCoarse &cd, double *phi, void *psi, hipStream_t s);

void launch_sweep(const SweepArgs &a, int precision, int exp_mode, bool currents, int nb, int np, int gb, int n_gb,
                  hipStream_t s);
void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
void launch_tally_bound(const DevProblem &d, const void *psi_in, hipStream_t s);
void launch_fill_real(void *p, int64_t n, int precision, hipStream_t s);
void launch_scale_real(void *p, int64_t n, int precision, const double *f, hipStream_t s);
void launch_scale_f64(double *p, int64_t n, const double *f, hipStream_t s);
void launch_prep_user(const DevProblem &d, const double *src_user, hipStream_t s);
void launch_source(const DevProblem &d, const double *phi, hipStream_t s);
void launch_finalize(const DevProblem &d, double *phi_internal, double *phi_user, double *partials, hipStream_t s);
void launch_fission_partials(const DevProblem &d, const double *phi, double *partials, hipStream_t s);
void launch_k_estimate(const DevProblem &d, const double *phi, double *partials, hipStream_t s);
void launch_eigen_update(const DevProblem &d, const double *partials, int mode, hipStream_t s);
void launch_norm_residual(const DevProblem &d, double *phi_new, const double *phi_old, double *partials, hipStream_t s);
void launch_psi_canon(const DevProblem &d, double *canon, void *psi, int to_canon, hipStream_t s);
void launch_psi_from_phi(const DevProblem &d, const double *phi_internal, void *psi, hipStream_t s);
void launch_permute_rows(const DevProblem &d, const double *src, double *dst, int to_user, hipStream_t s);
void launch_check_guess(const double *x, int64_t n, double *out2, hipStream_t s);

}  // namespace moc
