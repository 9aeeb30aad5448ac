/*
 * dfem.h -- C ABI of libmoc's DFEM-SN solver: discontinuous finite elements in space and
 * discrete ordinates in angle (paper Sec. 2.2, Eqs. DFEM_basis, DFEM_weak, DFEM_parts,
 * DFEM_upwind; GPU organisation of Sec. 3.3, Alg. DFEM_SN_sweep), on planar triangular
 * meshes, for AMD Instinct MI355X (gfx950).
 *
 * Every triangle is an element with the linear modal basis u_0 = 1, u_1 = (x - x_c)/L,
 * u_2 = (y - y_c)/L (centroid x_c, y_c; L = sqrt(area)). The angular variable is the
 * product quadrature of n_azim equally spaced azimuths phi_a = 2 pi (a + 1/2) / n_azim
 * and n_polar half-range Gauss-Legendre polar cosines (or the caller's); each in-plane
 * direction carries both polar hemispheres (weight 4 pi w_p / n_azim). A sweep solves,
 * for every direction, element and group, the element's 3x3 upwind system; all
 * directions advance together, one dependency level after another, and each element's
 * angular flux lives in a storage slot that is reused once every downstream element has
 * read it (Alg. DFEM_SN_sweep's compressed storage). With tiles (moc_sn_set_tiles) the
 * levels are taken tile by tile instead.
 *
 * Conventions are those of moc.h. Arrays of the solver are [T][G][3]: triangle (the
 * caller's triangle numbering), group, modal coefficient; FP64, row-major. Domains are
 * boxes; sides are vacuum or reflective (a reflective side feeds each direction the
 * mirrored direction's outgoing flux of the previous sweep).
 */
#ifndef DFEM_H
#define DFEM_H

#include "moc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct moc_sn_ctx moc_sn_ctx;

typedef struct {
    int32_t n_elements, n_directions, n_groups;
    int32_t n_levels;         /* dependency levels of the sweep (kernel launches per sweep) */
    int64_t n_tasks;          /* element-direction pairs per sweep */
    int64_t n_slots;          /* angular-flux storage slots (element-directions held at once) */
    int64_t n_boundary_faces;
    int64_t device_bytes;
    double setup_ms;
    int32_t tasks_per_thread; /* tasks one thread of a sweep step takes: the polar directions
                                 of one element and azimuth (n_polar), or 1 when a level does
                                 not consist of such runs */
    int32_t n_tiles;          /* tiles of the tiled schedule, 0 when sweeps run level by level */
    int32_t n_tile_levels;    /* tile levels (kernel launches per sweep) of the tiled schedule */
    int32_t max_inner_levels; /* most dependency levels inside one tile for one direction group */
    int32_t tile_lds_bytes;   /* LDS of one block of the tiled sweep */
    int64_t n_tile_slots;     /* storage slots of the tiled schedule (fluxes passed between tiles) */
} moc_sn_info;

/* Create a DFEM-SN context. mesh as for moc_create (box domain only); angles: n_azim (a
 * positive multiple of 4) and n_polar (1..4), optional polar_mu / polar_w; its spacing is
 * not used. xs as for moc_create. opts: precision (FP32 / FP64 local solves; tallies,
 * source, eigenvalue and norms are FP64), max_iter, check_every, device, n_threads.
 * Errors: MOC_EINVAL (as moc_create; a hexagonal domain; a boundary edge off the box),
 * MOC_ENOMEM, MOC_EHIP. */
int moc_sn_create(const moc_mesh *mesh, const moc_tracks *angles, const moc_xs *xs, const moc_options *opts,
                  moc_sn_ctx **out);
void moc_sn_destroy(moc_sn_ctx *ctx);

/* One sweep of every direction and group for emission moments source_dev (device
 * [T][G][3], per unit volume over all directions; the library applies 1/(4 pi)); writes
 * the scalar-flux moments phi_out_dev (device [T][G][3]). Reflective inflow comes from
 * the previous sweep (state carried between calls). Asynchronous on stream (NULL: the
 * context's). Errors: MOC_EINVAL (null pointer), MOC_EHIP. */
int moc_sn_sweep(moc_sn_ctx *ctx, const double *source_dev, double *phi_out_dev, void *stream);

/* Power iteration (or source iteration with an external source), cold start, as
 * moc_solve with F = sum_e area_e nuSigma_f phi_0 and the residual in the L2 norm of the
 * linear field. Synchronous. Errors: MOC_EINVAL (tol <= 0, null out), MOC_ENOCONV. */
int moc_sn_solve(moc_sn_ctx *ctx, double tol, moc_result *out);
int moc_sn_run_iterations(moc_sn_ctx *ctx, int32_t n, moc_result *out);

/* Scalar-flux moments of the last iteration (device [T][G][3]). */
int moc_sn_get_flux(moc_sn_ctx *ctx, double *phi_dev, void *stream);

/* External isotropic source moments (device [T][G][3], copied), or NULL for the
 * eigenvalue problem. */
int moc_sn_set_external_source(moc_sn_ctx *ctx, const double *q_dev);

int moc_sn_get_info(const moc_sn_ctx *ctx, moc_sn_info *info);

/* Sweep by tiles (same dependency order as Alg. DFEM_SN_sweep, scheduled in two tiers):
 * element_tile (host [n_elements], copied) assigns every element to one of n_tiles tiles.
 * For each direction group (the polar directions of one azimuth) the tiles are ordered by
 * their own dependencies (a tile feeds another through the faces between them) into tile
 * levels, one kernel launch each; a block takes one tile and direction group, copies what
 * its elements read into LDS and walks the tile's elements level by level, keeping the
 * fluxes read inside the tile in LDS; only fluxes read by another tile go through storage
 * slots. Convex tiles (for example the pin cells of a lattice) never depend on each other
 * in a cycle. The fluxes are the same as with level-by-level sweeps bit for bit (the
 * scalar flux is summed in direction order either way). n_tiles = 0 with element_tile =
 * NULL returns to level-by-level sweeps; a refused tiling leaves the previous schedule in
 * place. The LDS one block needs (moc_sn_info.tile_lds_bytes) grows with the tile's
 * elements and the groups: on the order of 370 bytes per element at 7 groups in FP32,
 * twice that in FP64. Errors: MOC_EINVAL (tile index out of range, an empty tile, tiles
 * whose dependencies form a cycle for some direction, a tile whose block needs more LDS
 * than the device gives one block (host-only contexts assume 160 KiB), n_tiles > 0 with
 * NULL element_tile or the reverse), MOC_ENOMEM, MOC_EHIP. Works on host-only contexts
 * too (the schedule is built and checked on the host). */
int moc_sn_set_tiles(moc_sn_ctx *ctx, int32_t n_tiles, const int32_t *element_tile);

/* Sweep timing with HIP events (moc_profile: sweeps, total, min and max ms). */
int moc_sn_set_profiling(moc_sn_ctx *ctx, int32_t enable);
int moc_sn_get_profile(moc_sn_ctx *ctx, moc_profile *out);

const char *moc_sn_last_error(const moc_sn_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DFEM_H */
