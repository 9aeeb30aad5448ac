// Device state and kernel launchers of the DFEM-SN solver (see dfem_kernels.hip).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace moc {

// inflow codes per (task, face), decided on the host in FP64
constexpr int kSnOutflow = -1;   // Omega . n >= 0: the face adds to the local matrix
constexpr int kSnVacuum = -3;    // inflow through a vacuum side: nothing enters
// >= 0: inflow from the upstream element's storage slot; <= -4: reflective inflow read
// from boundary entry (-4 - code)

struct DevSN {
    int T = 0, G = 0, M = 0, nd = 0, nsteps = 0, precision = 0;
    int tgroup = 1;          // consecutive tasks (the polar directions of one element and
                             // azimuth) taken by one thread of the sweep step
    int64_t ntask = 0, nslot = 0, nbnd = 0;
    std::vector<int64_t> step_off;   // host [nsteps + 1]
    // geometry, sweep precision
    void *mass = nullptr;    // [T][6] symmetric 3x3 (00 01 02 11 12 22)
    void *fmass = nullptr;   // [T][3][6] face matrices int_f u_j u_i
    void *fcpl = nullptr;    // [T][3][9] coupling int_f u_j (own) u_k (neighbour)
    void *nrm = nullptr;     // [T][3][2] outward unit normals
    void *gradw = nullptr;   // [T] area / L (streaming term of the slopes)
    void *sigt = nullptr;    // [T][G] Sigma_t of each element's material
    void *dirs = nullptr;    // [nd][3] (Omega_x, Omega_y, weight)
    double *area = nullptr;  // [T]
    double *massd = nullptr; // [T][9] FP64 mass matrices for the norms
    int *mat = nullptr;      // [T]
    double *sigs_m = nullptr, *nsf_m = nullptr, *chi_m = nullptr;
    // tasks (element, direction) sorted by level
    int *task_e = nullptr, *task_d = nullptr, *task_slot = nullptr;
    int *inflow = nullptr;   // [ntask][3]
    int *bwrite = nullptr;   // [ntask][3] boundary entry written, or -1
    void *psi = nullptr;     // [nslot][G][3]
    void *bnd[2] = {nullptr, nullptr};  // [nbnd][G][3], entry = boundary face * nd + direction
    void *q = nullptr;       // [T][G][3] per steradian
    double *phi_acc = nullptr;          // [T][G][3]
    int64_t nrun = 0;        // runs of tgroup tasks per sweep (run r = tasks r tgroup ...)
    void *run_acc = nullptr; // [nrun][G][3] scalar-flux contribution of each run (sweep precision)
    int *elem_off = nullptr; // [T + 1] runs of element e: elem_runs[elem_off[e] .. elem_off[e+1])
    int *elem_runs = nullptr;
    double *phi[2] = {nullptr, nullptr};
    double *qext = nullptr;
    double *partials = nullptr, *scal = nullptr;
};

struct SnStepArgs {
    const void *mass, *fmass, *fcpl, *nrm, *gradw, *sigt, *dirs, *q;
    const int *mat, *task_e, *task_d, *task_slot, *inflow, *bwrite;
    void *psi;
    const void *bnd_in;
    void *bnd_out;
    void *run_acc;
    int64_t k0, k1;
    int G;
    int tgroup;
};

void launch_sn_step(const SnStepArgs &a, int precision, hipStream_t s);
void launch_sn_gather(const DevSN &d, hipStream_t s);
void launch_sn_prep_user(const DevSN &d, const double *src, hipStream_t s);
void launch_sn_source(const DevSN &d, const double *phi, hipStream_t s);
void launch_sn_finalize(const DevSN &d, double *phi_internal, double *phi_user, double *partials, hipStream_t s);
void launch_sn_fission_partials(const DevSN &d, const double *phi, hipStream_t s);
void launch_sn_eigen_update(const DevSN &d, int mode, hipStream_t s);
void launch_sn_norm_residual(const DevSN &d, double *phi_new, const double *phi_old, hipStream_t s);
void launch_sn_fill(void *p, int64_t n, int precision, hipStream_t s);
void launch_sn_fill_f64(double *p, int64_t n, double v, hipStream_t s);
void launch_sn_scale(void *p, int64_t n, int precision, const double *f, hipStream_t s);
void launch_sn_scale_f64(double *p, int64_t n, const double *f, hipStream_t s);
void launch_sn_cold(double *phi, int64_t n, hipStream_t s);

// indices into DevSN::scal
enum { kSnK = 0, kSnKPrev = 1, kSnF = 2, kSnRes = 3, kSnDk = 4, kSnCount = 8 };
constexpr int kSnReduceBlocks = 256;

}  // namespace moc
