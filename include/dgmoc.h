/*
 * dgmoc.h -- C ABI of libmoc's DGMOC solver: the planar method of characteristics
 * extended to axially extruded 3D problems by a discontinuous Galerkin discretisation in z
 * (paper Sec. 2.1.1, Eqs. DGMOC_expansion, DGMOC_weak, DGMOC_weak_up; sweep organisation
 * of Sec. 3.2, Alg. DGMOC_sweep), for AMD Instinct MI355X (gfx950).
 *
 * The 3D domain is the planar mesh of moc.h stacked into n_planes axial planes. In every
 * plane the angular flux and the source are linear in z (Legendre basis 1 and xi on the
 * plane, xi = -1 at its bottom face and +1 at its top, the linear order the paper uses);
 * the flux entering through an axial face comes from the neighbouring plane (upwinding),
 * flat over each 2D element and direction. Along every 2D segment the two coefficients
 * obey a 2x2 linear ODE solved exactly (a 2x2 matrix exponential). A sweep runs the
 * upward directions plane by plane from the bottom, then the downward ones from the top;
 * every plane step is: driven flux, ray tracing of the plane, scalar-flux restoration,
 * axial face flux for the next plane.
 *
 * Conventions are those of moc.h (status codes, host/device pointers, region numbering,
 * one context per device, calls on one context serialised by the caller). Arrays of the
 * extruded problem are [n_planes][R][G][2]: plane, user region, group, Legendre moment
 * (0: plane average; 1: coefficient of xi), FP64, row-major.
 */
#ifndef DGMOC_H
#define DGMOC_H

#include "moc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct moc_dg_ctx moc_dg_ctx;

/* Axial description of an extruded problem. */
typedef struct {
    int32_t n_planes;               /* >= 1 */
    const double *dz;               /* host [n_planes] plane heights in cm, bottom to top, each > 0 */
    const int32_t *plane_material;  /* host [n_planes][R] material of each (plane, region), or NULL:
                                       mesh->region_material in every plane */
    int32_t bc_bottom, bc_top;      /* MOC_BC_VACUUM or MOC_BC_REFLECTIVE */
    int32_t angle_block;            /* track angles swept together (Alg. DGMOC_sweep's angle blocks);
                                       0: all angles in one block. Smaller blocks need less device
                                       memory for the face fluxes, in exchange for more launches */
} moc_axial;

typedef struct {
    int32_t n_planes, n_blocks, angles_per_block;
    int32_t group_batch;      /* groups per sweep wavefront */
    int64_t n_updates;        /* per sweep: 2D segments x 2 senses x n_polar x 2 wards x G x n_planes */
    int64_t device_bytes;     /* device memory held by the context */
    double setup_ms;          /* host setup time of moc_dg_create */
} moc_dg_info;

/* Create a DGMOC context. mesh, tracks and xs are as for moc_create (Sec. 3.1 tracking;
 * the mesh's region_material must be valid and is the default plane map); axial adds
 * the planes. opts as for moc_create, with these DGMOC defaults when left 0:
 * tally_slots 256, group_batch 2 (allowed: 1, 2, 4). exp_mode, window_steps,
 * lane_stagger and batch_order apply to the shared track packing only. The context
 * starts cold: scalar flux moments (1, 0), k = 1, zero boundary and face fluxes.
 * Errors: MOC_EINVAL (as moc_create; n_planes < 1, dz <= 0, a plane material out of
 * range, bad bc, angle_block < 0, group_batch not 1, 2 or 4), MOC_ENOMEM, MOC_EHIP. */
int moc_dg_create(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs, const moc_axial *axial,
                  const moc_options *opts, moc_dg_ctx **out);
void moc_dg_destroy(moc_dg_ctx *ctx);

/* One transport sweep (both wards, all planes and angle blocks) for a given isotropic
 * emission density: source_dev device [n_planes][R][G][2] (n/cm^3/s per unit volume over all
 * directions; moment 1 is the xi coefficient; the library applies 1/(4 pi)). Writes the
 * scalar-flux moments to phi_out_dev (device, same layout). Enqueued on stream (NULL:
 * the context's stream), asynchronous. Reads and updates the radial boundary fluxes and
 * the bottom-face fluxes kept by the context (state carried between calls).
 * Errors: MOC_EINVAL (null pointer), MOC_EHIP. */
int moc_dg_sweep(moc_dg_ctx *ctx, const double *source_dev, double *phi_out_dev, void *stream);

/* Power iteration (or, with an external source set, source iteration with k = 1) to
 * tol: every iteration sweeps once with the previous iterate's emission (Eq. MGNTE,
 * isotropic scattering, applied to both moments), updates
 * k <- k sum V h nuSigma_f phi_0 (new) / (old), normalises that sum to 1, and stops when
 * the relative change of the flux in the L2 norm of the linear field (weights V h for
 * moment 0, V h / 3 for moment 1) and |dk| are both below tol. Cold start every call.
 * Synchronous. moc_result as for moc_solve. Errors: MOC_EINVAL (tol <= 0, null out),
 * MOC_ENOCONV (max_iter reached; out is filled), MOC_EHIP. */
int moc_dg_solve(moc_dg_ctx *ctx, double tol, moc_result *out);

/* Exactly n iterations from the cold start (timing); out as for moc_dg_solve. */
int moc_dg_run_iterations(moc_dg_ctx *ctx, int32_t n, moc_result *out);

/* Scalar-flux moments of the last iteration into phi_dev (device [n_planes][R][G][2]). */
int moc_dg_get_flux(moc_dg_ctx *ctx, double *phi_dev, void *stream);

/* External isotropic source moments q_dev (device [n_planes][R][G][2], copied), or NULL
 * to return to the eigenvalue problem. Errors: MOC_EINVAL only for a failed copy. */
int moc_dg_set_external_source(moc_dg_ctx *ctx, const double *q_dev);

int moc_dg_get_info(const moc_dg_ctx *ctx, moc_dg_info *info);

/* Sweep timing with HIP events around every moc_dg_sweep / iteration sweep while enabled
 * (moc_profile: sweeps, total, min and max ms per sweep; cmfd fields zero). */
int moc_dg_set_profiling(moc_dg_ctx *ctx, int32_t enable);
int moc_dg_get_profile(moc_dg_ctx *ctx, moc_profile *out);

/* Message of the last failed call on ctx (NULL: of the last failed moc_dg_create on this
 * thread). Valid until the next call on ctx. */
const char *moc_dg_last_error(const moc_dg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DGMOC_H */
