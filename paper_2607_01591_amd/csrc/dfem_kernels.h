// Device state and kernel launchers of the DFEM-SN solver (see dfem_kernels.hip).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace moc {

// inflow codes per (task, face), decided on the host in FP64
constexpr int kSnOutflow = -1;   // Omega . n >= 0: the face adds to the local matrix
constexpr int kSnVacuum = -3;    // inflow through a vacuum side: nothing enters
// tiled schedule (codes of its own task records): kSnLocalFlag | l = interior inflow from
// the tile's LDS flux of its element l; kSnExtFlag | j = interior inflow from staged entry
// j (another tile's storage slot); -4 - j = reflective inflow from staged entry j (the
// boundary buffer)
constexpr int kSnLocalFlag = 1 << 30;
constexpr int kSnExtFlag = 1 << 29;
constexpr int kSnRecInts = 9;           // item record: tile element, LDS slot, 3 inflow codes,
                                        // 3 boundary writes, storage slot (polar direction 0)
constexpr int kSnElemHead = 13;         // staged element data: mass 6, gradw 1, normals 6,
                                        // then one face block per face (9, 6 or 0 reals)
// regions of a tile block's LDS (byte offsets in SnTileArgs::lds_off)
enum { kSnLdsPsi = 0, kSnLdsElem, kSnLdsSq, kSnLdsExt, kSnLdsDir, kSnLdsTask, kSnLdsElemId, kSnLdsFine, kSnLdsCount };
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
    int ndg = 0;             // direction groups (runs of tgroup directions of one azimuth)
    void *run_acc = nullptr; // [ndg][T][G][3] scalar-flux contribution of each run (sweep precision)
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
    int ndg;
    int T;
};

// one launch of the tiled schedule: blocks take the tile tasks tt0, tt0 + 1, ...; the
// tasks of level j inside tile task tt are tt_task[tt] + [fine_off[j], fine_off[j + 1]) for
// j in [tt_fine[tt], tt_fine[tt + 1] - 1) (each tile task stores its levels' starts and the
// end of its last level)
struct SnTileArgs {
    const int64_t *tt_task;
    const int *tt_fine;
    const int *fine_off;
    const int *tt_tile, *tt_dg;        // tile and direction group of each tile task
    const int *tile_off, *tile_elems;  // elements of each tile (ascending)
    const int *ext_off, *ext_src;      // staged inflow entries of each tile task: a storage
                                       // slot (>= 0) or a boundary code (<= -4)
    const int *rec;                    // item records (item = tile task element, task / tgroup)
    int64_t tt0;
    int el_stride;                     // reals of one item's staged element data
    unsigned lds_off[kSnLdsCount];
};

// device arrays of the tiled schedule (own task order, slots and codes)
struct DevSNTiles {
    int n_tiles = 0, n_levels = 0;      // tiles; tile levels (launches per sweep)
    int max_tile = 0;                   // elements of the largest tile
    int max_inner = 0;                  // most dependency levels inside one tile task
    size_t lds_bytes = 0;               // LDS of one block
    int64_t nslot = 0;
    std::vector<int64_t> lev_off;       // host [n_levels + 1]: tile tasks of each tile level
    unsigned lds_off[kSnLdsCount] = {};
    int max_live = 0;                   // LDS flux slots of one tile task
    int el_stride = 0;                  // reals of one item's staged element data
    int *rec = nullptr;                 // item records [item][kSnRecInts]
    int64_t *tt_task = nullptr;
    int *tt_fine = nullptr, *fine_off = nullptr, *tt_tile = nullptr, *tt_dg = nullptr;
    int *tile_off = nullptr, *tile_elems = nullptr, *ext_off = nullptr, *ext_src = nullptr;
    void *psi = nullptr;                // [nslot][G][3]
};

void launch_sn_step(const SnStepArgs &a, int precision, hipStream_t s);
void launch_sn_gather(const DevSN &d, hipStream_t s);
void launch_sn_tile(const SnStepArgs &a, const SnTileArgs &t, int nblocks, size_t lds_bytes, int precision, hipStream_t s);
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
