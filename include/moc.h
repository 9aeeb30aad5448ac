/*
 * moc.h -- C ABI of libmoc: flat-source planar Method of Characteristics on
 * unstructured 2D triangular meshes, for AMD Instinct MI355X (gfx950).
 *
 * The library solves the steady multigroup k-eigenvalue (or fixed-source) transport
 * equation with isotropic scattering (paper Sec. 2, Eq. MGNTE and Eq. MGNTE_element)
 * by the planar method of characteristics (Sec. 2.1): every mesh region is a flat-
 * source region, straight cyclic tracks are laid on the bounding box of the domain
 * and intersected with the mesh (Sec. 3.1), and along each segment the angular flux
 * is attenuated by Eq. MOC_sol; the scalar flux is the angular integral of the
 * segment-averaged flux.
 *
 * Conventions (all entry points):
 *   - Every function returns MOC_OK (0) or an error code; nothing throws across the
 *     boundary. moc_last_error() describes the last failure.
 *   - "host" pointers are ordinary CPU memory; they are only read during the call and
 *     may be freed by the caller on return (the library copies what it keeps).
 *   - "device" pointers are caller-owned HIP device allocations on the context's
 *     device, contiguous, in the layout stated; the library never frees them.
 *   - Region-indexed arrays [R][G] are in the caller's region numbering
 *     (row-major, group fastest). Groups are numbered from fastest (0) to slowest.
 *   - Scattering matrices are sigma_s[m][g_from][g_to].
 *   - Calls on one context must be serialised by the caller; separate contexts are
 *     independent. A context is bound to the HIP device named in its options.
 */
#ifndef MOC_H
#define MOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MOC_OK 0
#define MOC_EINVAL 1   /* invalid argument: bad topology, Sigma_t <= 0, null pointer ... */
#define MOC_ENOMEM 2   /* host or device allocation failed */
#define MOC_EHIP 3     /* a HIP runtime call or kernel launch failed */
#define MOC_ENOCONV 4  /* moc_solve reached max_iter; the result is still filled in */
#define MOC_ESTATE 5   /* call not valid in the context's current state */

/* boundary conditions, per domain side */
#define MOC_BC_VACUUM 0
#define MOC_BC_REFLECTIVE 1

/* domain shapes */
#define MOC_DOMAIN_BOX 0      /* axis-aligned rectangle box[0..3] = x0, y0, x1, y1 */
#define MOC_DOMAIN_HEXAGON 1  /* regular hexagon centred in box, flats parallel to x */

/* sweep precision */
#define MOC_PREC_F32 0   /* FP32 sweep; FP64 source, eigenvalue, norms and tallies */
#define MOC_PREC_F64 1   /* FP64 everywhere (same kernels instantiated in double) */

/* evaluation of the segment update of Eq. MOC_sol in the FP32 sweep (the FP64 sweep
 * always forms (psi - qhat)(1 - e^-tau) with expm1) */
#define MOC_EXP_POLY 0   /* default: 1 - e^-tau as the larger of two lower bounds, a degree-4
                            Taylor polynomial and the hardware exponential lowered by 4 units
                            in the last place: relative error <= 2.7e-6 for every tau */
#define MOC_EXP_TABLE 1  /* linear interpolation in a table of (1 - e^-x)/x */
#define MOC_EXP_LIBM 2   /* device libm expm1f */
#define MOC_EXP_DIFF 3   /* fastest: e = e^-tau from the hardware exponential (within 0.8 units
                            in the last place on gfx950) and the increment (psi - qhat)(1 - e) as
                            one fused multiply-add t - t e. Its error is the exponential's
                            absolute error, about 5e-8 / tau relative per segment: accurate where
                            regions are crossed by many segments of ordinary optical thickness,
                            not on meshes with sliver regions (tau ~ 1e-5 gives 1e-2) */

/* moc_result.flags */
#define MOC_FLAG_FELL_BACK_TO_COLD 1  /* the initial guess was rejected; cold start used */
#define MOC_FLAG_FIXED_SOURCE 2       /* an external source was set: source iteration */

typedef struct moc_ctx moc_ctx;

/* Mesh: triangles are the elements; a region (flat-source region, Sec. 2.1) is a set
 * of triangles (one triangle per region is the usual case). */
typedef struct {
    int32_t n_vertices;
    const double *xy;              /* host [n_vertices][2] */
    int32_t n_triangles;
    const int32_t *tri;            /* host [n_triangles][3], counter-clockwise */
    const int32_t *tri_region;     /* host [n_triangles], values in [0, n_regions) */
    int32_t n_regions;
    const int32_t *region_material;/* host [n_regions], values in [0, n_materials) */
    int32_t domain;                /* MOC_DOMAIN_* */
    double box[4];                 /* bounding box x0, y0, x1, y1 of the domain */
    double hex_apothem;            /* hexagon: centre-to-flat distance */
    int32_t bc[6];                 /* box: x = x0, x = x1, y = y0, y = y1; hexagon: 6 sides */
} moc_mesh;

/* Tracking parameters (Sec. 3.1, modular rays on the whole-domain bounding box). */
typedef struct {
    int32_t n_azim;         /* azimuthal directions over [0, 2 pi), a positive multiple of 4 */
    int32_t n_polar;        /* polar angles per hemisphere, 1..4 */
    double spacing;         /* nominal track spacing in cm (the corrected spacing is <= it) */
    const double *polar_mu; /* host [n_polar] polar cosines, or NULL for half-range Gauss-Legendre */
    const double *polar_w;  /* host [n_polar] weights summing to 1 (required with polar_mu) */
} moc_tracks;

/* Multigroup macroscopic cross sections per material (Eq. MGNTE, isotropic part). */
typedef struct {
    int32_t n_materials;
    int32_t n_groups;
    const double *sigma_t;    /* host [M][G], each > 0 */
    const double *sigma_s;    /* host [M][G][G], from -> to */
    const double *nu_sigma_f; /* host [M][G] */
    const double *chi;        /* host [M][G] */
} moc_xs;

typedef struct {
    int32_t precision;   /* MOC_PREC_* */
    int32_t exp_mode;    /* MOC_EXP_* (FP32 sweep only) */
    int32_t max_iter;    /* moc_solve iteration limit (<= 0: 10000) */
    int32_t device;      /* HIP device ordinal; negative: host-only context (tracking,
                            volumes, quadrature and info only; device calls return
                            MOC_ESTATE) */
    int32_t check_every; /* moc_solve reads (k, residual) back every this many iterations (<= 0: 1) */
    int32_t n_threads;   /* host threads for tracking (<= 0: all hardware threads) */
    double window_cm;    /* tally window length along the tracks in cm (<= 0: about 32
                            segments per window) */
    int32_t tally_slots; /* maximum distinct regions per tally window, 64..256 (0: 256) */
    int32_t group_batch; /* groups per sweep wavefront: 1, 2, 4, 7, 8 or 11 (0: chosen from G) */
    int32_t window_steps;/* > 0: tally windows of this many segments per track instead of a
                            fixed length along the tracks (lanes stay busy, slots grow) */
    int32_t lane_stagger;/* S > 1: lane l of every tally window starts (l mod S) steps late,
                            so lanes at one step sit at different places along their tracks
                            and fewer of them add to the same LDS tally row at once (costs up
                            to S - 1 padding steps per window); 1: none; 0: library default (2) */
    int32_t batch_order; /* 0: workgroups in batch order; 1: each of the 8 XCDs (own L2)
                            sweeps one contiguous range of batches */
} moc_options;

typedef struct {
    double k;            /* eigenvalue (1 in fixed-source mode) */
    int32_t iterations;
    double residual;     /* ||sqrt(V)(phi_n - phi_n-1)|| / ||sqrt(V) phi_n|| of the last iteration */
    double dk;           /* |k_n - k_n-1| of the last iteration */
    double wall_ms;      /* host wall time of the solve */
    int32_t flags;       /* MOC_FLAG_* */
    int32_t sweeps;      /* transport sweeps performed, including warm-start boundary sweeps */
} moc_result;

typedef struct {
    int32_t n_regions, n_groups, n_materials, n_polar, n_angles;
    int32_t n_tracks;          /* T: tracks that cross the domain */
    int64_t n_segments;        /* S: 2D segments after merging */
    int64_t n_updates;         /* U = 2 * P * G * S per sweep */
    int64_t n_padded_steps;    /* segment slots the sweep walks (incl. padding), per sense */
    int32_t n_batches;         /* 64-track wavefront batches */
    int64_t n_windows;         /* tally windows over all batches */
    int64_t n_window_slots;    /* sum of distinct regions over all windows (tally flushes per
                                  group and sense) */
    double window_cm;          /* tally window length used */
    int32_t max_window_slots;  /* largest slot count of any window */
    double setup_ms;           /* host setup time of moc_create */
    int64_t device_bytes;      /* device memory held by the context */
    int32_t precision;
    int32_t lane_stagger;      /* lane stagger of the tally windows in use */
} moc_info;

/* Device-time profile of the sweep kernel and of the CMFD steps, from HIP events recorded
 * on the stream they are launched on (enabled by moc_set_profiling). */
typedef struct {
    int64_t sweeps;       /* sweep kernel launches timed since profiling was enabled */
    double sweep_ms;      /* total device time of those launches */
    double sweep_ms_min;  /* shortest launch */
    double sweep_ms_max;  /* longest launch */
    int64_t cmfd_steps;   /* CMFD steps timed (homogenisation, coarse solve, prolongation) */
    double cmfd_ms;       /* their total device time */
} moc_profile;

/* Convergence controls of the CMFD coarse solve (moc_set_coarse_mesh). Zero fields take
 * the defaults. */
typedef struct {
    double tol;          /* largest relative change of k and of the coarse flux that ends
                            the coarse power iteration; each step uses the smaller of tol and
                            a tenth of the last power iteration's residual, and the BiCGSTAB
                            solves stop at a tenth of that relative residual (default 1e-3) */
    double shift;        /* Wielandt shift k_s = k (1 + shift), applied once k has settled
                            and then kept for the step (default 0.02; negative: never shift) */
    int32_t max_outer;   /* coarse power iterations per CMFD step (default 8) */
    int32_t max_inner;   /* BiCGSTAB iterations per coarse linear solve (default 200) */
    int32_t coarse_blocks; /* coarse solve on one 1024-thread workgroup (1) or on a
                              cooperative grid of this many 256-thread blocks (2..256);
                              0: one workgroup up to 4096 unknowns (cells x groups), else
                              one block per 256 unknowns */
} moc_cmfd_options;

/* Coarse mesh state (moc_get_coarse_info); all zero when no coarse mesh is set. */
typedef struct {
    int32_t n_cells;
    int32_t n_surfaces;    /* coarse surfaces crossed by some track, boundary ones included */
    int64_t n_crossings;   /* crossing entries in the packed segment stream */
    double setup_ms;       /* host time of moc_set_coarse_mesh */
    int32_t last_outer;    /* coarse power iterations of the last CMFD step */
    int32_t last_inner;    /* BiCGSTAB iterations of the last CMFD step (all solves) */
    double last_k;         /* coarse eigenvalue of the last CMFD step */
} moc_coarse_info;

/* Build a solver context (host setup in C++: mesh half-edge structure, cyclic track
 * laydown, ray tracing by mesh walk, segment merging, boundary links, track volumes,
 * device packing). All inputs are copied. Errors: MOC_EINVAL (inconsistent topology,
 * clockwise triangle, non-manifold edge, a region without triangles, material index
 * out of range, Sigma_t <= 0, n_azim % 4 != 0, n_polar outside 1..4, reflective hexagon,
 * mesh not covering the domain), MOC_ENOMEM, MOC_EHIP. */
int moc_create(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs,
               const moc_options *opts, moc_ctx **out);

/* Release the context and every device buffer it owns. NULL is allowed. */
void moc_destroy(moc_ctx *ctx);

/* One transport sweep (Eq. MOC_sol on every segment, direction, polar angle and group)
 * for a given isotropic emission density. source_dev: device FP64 [R][G], neutrons per
 * cm^3 per s over all directions (the library divides by 4 pi). scalar_flux_out_dev:
 * device FP64 [R][G] receives phi = 4 pi qhat + T / (Sigma_t V). Enqueued on the HIP
 * stream `stream` (NULL = the context's own stream); returns without waiting. Reads the
 * context's incoming boundary angular fluxes and stores the outgoing ones as the next
 * sweep's incoming fluxes (reflective sides), so consecutive calls iterate. */
int moc_sweep(moc_ctx *ctx, const double *source_dev, double *scalar_flux_out_dev, void *stream);

/* Power iteration (or source iteration with an external source) to `tol`: the
 * k-eigenvalue problem of Eq. MGNTE (Sec. 2; k_eff is the largest eigenvalue, found by
 * repeated transport sweeps, Sec. 2.1, each applying Eq. MOC_sol to every segment, until
 * convergence). Each iteration: source from the previous flux (Jacobi in energy),
 * one sweep, k <- k sum V nuSigma_f phi_new / sum V nuSigma_f phi_old, normalisation to
 * sum V nuSigma_f phi = 1 (FP64 on the device). Residual = ||sqrt(V)(phi_n - phi_n-1)||_2 /
 * ||sqrt(V) phi_n||_2 over all (region, group); stops when the residual and |dk| are both
 * below tol. Synchronous on the context's stream. Starts from the initial guess if one is
 * set (used once), else from phi = 1, k = 1, psi = 0. Returns MOC_ENOCONV at max_iter with
 * `out` filled in; MOC_EINVAL if tol <= 0 or out is NULL. */
int moc_solve(moc_ctx *ctx, double tol, moc_result *out);

/* Exactly n iterations of the moc_solve loop (same start rules) with a single
 * read-back of (k, residual) at the end, for timing. `out` holds the last iterate's
 * values. Returns MOC_OK after n iterations. */
int moc_run_iterations(moc_ctx *ctx, int n, moc_result *out);

/* Initial guess for the next moc_solve (the state the power iteration of Eq. MGNTE starts
 * from): phi0_dev device FP64 [R][G] (required, any scale; copied); k0 > 0, or k0 <= 0 to
 * estimate it as sum V nuSigma_f phi0 / sum V Sigma_a phi0; psi_b0_dev device FP64
 * [T][2][P][G] incoming boundary fluxes in canonical track order (copied), or NULL: then
 * psi starts at phi0 / 4 pi of the region where each track-sense enters and two transport
 * sweeps with the source frozen at (phi0, k0) make it consistent with the guess before the
 * iteration starts (counted in moc_result.sweeps). The solver owns the fallback, which is
 * not an error: a guess with a non-finite or negative entry, or all zeros, is not used,
 * and a guess whose residual, at any of its iterations 2 to 10, exceeds the first residual
 * of a cold start is abandoned for a cold restart (the first iteration of a guess also
 * relaxes its boundary fluxes and k, so it is not judged; the cold start's first residual is
 * measured by one cold iteration when not yet known for the current cross sections,
 * source mode and coarse mesh, and recorded by every cold-started solve); either way
 * moc_solve cold-starts and sets MOC_FLAG_FELL_BACK_TO_COLD, and moc_result.sweeps counts
 * every sweep made. Errors: MOC_EINVAL for a null phi0_dev. */
int moc_set_initial_guess(moc_ctx *ctx, const double *phi0_dev, double k0, const double *psi_b0_dev);

/* Copy the current scalar flux (the phi of Eq. MGNTE after the last sweep or iteration;
 * device FP64 [R][G], user region order) to phi_dev on `stream` (NULL: the context's
 * stream). Errors: MOC_EINVAL (null pointer), MOC_ESTATE (host-only context). */
int moc_get_flux(moc_ctx *ctx, double *phi_dev, void *stream);

/* Incoming boundary angular fluxes psi_in of Eq. MOC_sol at the start of every track
 * (Sec. 2.1; reflective sides feed them from the linked track's exit, vacuum sides hold 0),
 * device FP64 [T][2][P][G]; tracks in canonical order
 * (angle index ascending, then perpendicular coordinate -sin(phi) x + cos(phi) y
 * ascending), sense 0 = along (cos phi, sin phi). Get converts from the sweep precision;
 * set rounds to it. */
int moc_get_boundary_flux(moc_ctx *ctx, double *psi_dev, void *stream);
int moc_set_boundary_flux(moc_ctx *ctx, const double *psi_dev, void *stream);

/* Register a device FP64 [T][2][P][G] buffer that every following sweep fills with the
 * outgoing angular flux of each track-sense (NULL disables). For tests and diagnostics. */
int moc_set_exit_flux_buffer(moc_ctx *ctx, double *psi_exit_dev);

/* Fixed-source mode: q_dev device FP64 [R][G] external emission density (copied), or
 * NULL to return to eigenvalue mode. In fixed-source mode moc_solve iterates
 * s = Sigma_s^T phi + chi F + q with k = 1 and no normalisation. */
int moc_set_external_source(moc_ctx *ctx, const double *q_dev);

/* Replace the cross sections and the region -> material map of an existing context
 * without re-tracking (same mesh, same number of groups and materials). region_material
 * host [R] (user order); xs host arrays as in moc_create. Clears any external source and
 * pending initial guess. Errors: MOC_EINVAL (sizes differ, Sigma_t <= 0, bad material). */
int moc_set_materials(moc_ctx *ctx, const int32_t *region_material, const moc_xs *xs);

/* CMFD acceleration (Sec. 2.1.2, Alg. MOCHFEM_CMFD, its radial part): region_cell host
 * int32 [R] (user region order) assigns every region to one of n_cells coarse cells;
 * every cell must hold at least one region. From then on each sweep also tallies the net
 * current across every coarse surface a track crosses (the packed segment stream is
 * rebuilt with a crossing entry at every change of coarse cell and at both ends of every
 * track), and in eigenvalue mode every power iteration is followed by a CMFD step on the
 * device: flux-volume homogenisation onto the cells, diffusion couplings Dhat from the
 * cell geometry and Dtilde from the sweep's currents (Dhat = 0 on the domain boundary),
 * the coarse eigenproblem, and rescaling of the fine flux and of the incoming boundary
 * fluxes by each cell's ratio of new to homogenised flux; k comes from the coarse
 * problem. The converged answer is that of the plain power iteration. Fixed-source mode
 * is not accelerated. opts may be NULL (defaults). n_cells <= 0 or region_cell NULL
 * removes the coarse mesh. Host-only contexts set up the surfaces and packing only.
 * Errors: MOC_EINVAL (cell index out of range, an empty cell, exp_mode other than 0 with
 * FP32, too many regions plus surfaces for the segment key). */
int moc_set_coarse_mesh(moc_ctx *ctx, int32_t n_cells, const int32_t *region_cell,
                        const moc_cmfd_options *opts);
int moc_get_coarse_info(moc_ctx *ctx, moc_coarse_info *info);

/* Net currents of the last sweep across the coarse surfaces: cells host int32
 * [n_surfaces][2] receives each surface's cells (a, b), a < b, or (a, -1) for the part of
 * cell a's boundary on the domain boundary; current host FP64 [n_surfaces][G] the net
 * current from a to b (out of the domain for b = -1), integrated over the surface, with
 * the same weights as the flux tally. Either pointer may be NULL; current needs a device
 * context. Errors: MOC_ESTATE without a coarse mesh. */
int moc_get_surface_currents(moc_ctx *ctx, int32_t *cells, double *current);

/* Region containing each of n points (host xy [n][2]; host out [n] user region ids, -1
 * outside the mesh); a point on a shared edge gets one of the adjacent regions. */
int moc_locate_points(moc_ctx *ctx, const double *xy, int64_t n, int32_t *region_out);

/* Area-weighted centroid of every region (host [R][2], user order). */
int moc_get_centroids(const moc_ctx *ctx, double *xy_out);

int moc_get_info(const moc_ctx *ctx, moc_info *info);

/* Enable (non-zero) or disable timing of every sweep kernel launch with a pair of HIP
 * events on its stream; enabling resets the counters. moc_get_profile waits for the
 * timed launches to finish and reports them. */
int moc_set_profiling(moc_ctx *ctx, int enable);
int moc_get_profile(moc_ctx *ctx, moc_profile *out);

/* Track-estimated region volumes V_r (host FP64 [R], user order). */
int moc_get_volumes(const moc_ctx *ctx, double *V_host);

/* Tracking dump for tests (host arrays sized from moc_get_info): angle [T],
 * endpoints [T][4] (x0 y0 x1 y1 along sense 0), offsets [T+1], then the merged
 * segments region [S] (user ids) and length [S] in double, and links [T][2]
 * (destination track*2+sense, or -1 for vacuum). Any pointer may be NULL. */
int moc_get_tracks(moc_ctx *ctx, int32_t *angle, double *endpoints, int64_t *offsets,
                   int32_t *seg_region, double *seg_length, int32_t *links);

/* Packed sweep layout of a host-only context (MOC_ESTATE otherwise), for tests: batch
 * window ranges [n_batches + 1] and angles [n_batches]; per window: first entry,
 * steps, first slot-table entry and slot count [n_windows]; slot table (internal region
 * ids) [n_window_slots]; per entry [n_padded_steps]: length and key = (internal region
 * << 9) | slot; the user id of each internal region [n_regions]. Entries of a window
 * are [step][64 lanes]. Any pointer may be NULL. */
int moc_get_packing(const moc_ctx *ctx, int64_t *batch_win, int32_t *batch_angle,
                    int64_t *win_entry_off, int32_t *win_nsteps, int64_t *win_tab_off,
                    int32_t *win_nslots, int32_t *win_tab, double *seg_len, uint32_t *seg_key,
                    int32_t *user_of_internal);

/* Quadrature actually used: per track angle phi, delta, weight [n_angles]; polar
 * mu, weight [n_polar]. Any pointer may be NULL. */
int moc_get_quadrature(const moc_ctx *ctx, double *phi, double *delta, double *w_azim,
                       double *mu, double *w_polar);

/* Description of the last error on this context (ctx NULL: the calling thread's last
 * moc_create failure). Valid until the next call on the same context or thread. */
const char *moc_last_error(const moc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MOC_H */
