// Device state and kernel launchers of the DGMOC solver (see dg_kernels.hip for layouts).
#pragma once

#include "moc_kernels.h"

namespace moc {

// Arguments of one plane's driven-flux step (one ward, one angle block).
struct DgDrivenArgs {
    const void *sigt;     // Real [R][Gp] Sigma_t of the plane (padded groups: 1)
    const void *q;        // Real [R][Gp][2] source moments per steradian of the plane
    void *face;           // Real [2 NAb][P][R][Gp] raw face tallies of the previous plane; zeroed here
    const void *bot;      // Real [2 NA][P][R][Gp] face flux through the bottom (mode 2)
    const void *inv_va;   // Real [NA][R] 1 / (per-angle track area), 0 where no track passes
    void *drv;            // Real [2 NAb][R][n_gb][P][gb][2] driven flux out
    int mode;             // face flux entering: 0 none, 1 face tallies * inv_va, 2 bot
    int a0, nab, R, P, Gp, gb, n_gb;
    double kap[kMaxPolar];  // mu_p / h of the plane
    double sgn;             // +1 upward ward, -1 downward ward (mirrored xi)
};

// Arguments of one plane's ray tracing (one ward, one angle block).
struct DgSweepArgs {
    const void *segs;
    const int64_t *batch_win, *win_entry_off, *win_tab_off;
    const int *win_nsteps, *win_nslots, *win_tab;
    int cap;
    const int *batch_angle;
    int b0, a0;              // first batch and first track angle of the block
    const void *sigt;        // Real [R][Gp] of the plane
    const void *drv;         // Real [2 NAb][R][n_gb][P][gb][2]
    const void *psi_in;      // Real [2 senses][P][2][Gp][nslots] of the plane and ward
    void *psi_out;
    const int *link;
    const unsigned char *fed;
    const void *wdir;        // Real [NA][P] direction weight times delta_a
    const void *dlt;         // Real [NA]
    const void *inv_sin;     // Real [P]
    double kap[kMaxPolar];
    double sgn;
    double *tally;           // [R][Gp][2] of the plane
    void *face;              // Real [2 NAb][P][R][Gp]
    int nslots, Gp, R, n_gb;
};

struct DevDG {
    int Nz = 0, nab = 0, n_blocks = 0, gb = 4, n_gb = 2, Gp = 8;
    int bc_bot = 0, bc_top = 0;
    std::vector<double> dz;                  // [Nz] host
    std::vector<int> blk_angle0, blk_batch0; // [n_blocks + 1] host
    double mu[kMaxPolar] = {0, 0, 0, 0};
    int *mat3 = nullptr;      // [Nz][R] internal regions
    double *hV = nullptr;     // [Nz][R] V_r h_z
    void *sigt3 = nullptr;    // Real [Nz][R][Gp]
    void *q3 = nullptr;       // Real [Nz][R][Gp][2]
    void *drv = nullptr;
    void *face = nullptr;
    void *bot = nullptr;      // only with a reflective bottom
    void *inv_va = nullptr;
    void *wdir = nullptr, *dlt = nullptr;
    double *tally = nullptr;  // [Nz][R][Gp][2]
    double *phi[2] = {nullptr, nullptr};  // [Nz][R][G][2] internal
    void *psi[2] = {nullptr, nullptr};    // Real [2 wards][Nz][2][P][2][Gp][nslots]
    double *qext = nullptr;   // [Nz][R][G][2] internal, emission density
    int64_t psi_count = 0, face_count = 0, bot_count = 0;
};

void launch_dg_driven(const DgDrivenArgs &a, int precision, hipStream_t s);
void launch_dg_store_bottom(const DgDrivenArgs &a, int precision, hipStream_t s);
void launch_dg_sweep(const DgSweepArgs &a, int precision, int nb, int np, int gb, hipStream_t s);
void launch_dg_prep_user(const DevProblem &d, const DevDG &g, const double *src_user, hipStream_t s);
void launch_dg_source(const DevProblem &d, const DevDG &g, const double *phi, hipStream_t s);
void launch_dg_finalize(const DevProblem &d, const DevDG &g, double *phi_internal, double *phi_user, double *partials,
                        hipStream_t s);
void launch_dg_fission_partials(const DevProblem &d, const DevDG &g, const double *phi, double *partials, hipStream_t s);
void launch_dg_norm_residual(const DevProblem &d, const DevDG &g, double *phi_new, const double *phi_old, double *partials,
                             hipStream_t s);
void launch_dg_cold_flux(const DevDG &g, double *phi, int64_t n_cells, hipStream_t s);
void launch_dg_permute(const DevProblem &d, const DevDG &g, const double *src, double *dst, int to_user, hipStream_t s);

}  // namespace moc
