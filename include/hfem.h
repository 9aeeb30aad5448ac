/*
 * hfem.h -- C ABI of libmoc's coarse-mesh diffusion HFEM solver (hybrid finite elements,
 * i.e. the variational nodal method: paper Sec. 2.1.2, Eqs. HFEM_functional,
 * HFEM_weak_form, HFEM_flux_expansion, HFEM_current_expansion, HFEM_flux_response), with
 * the GPU organisation of Sec. 3.1: a preassembly that builds and inverts the reaction
 * matrix and then the response matrix of every node and group (batched, FP64), and a
 * solution phase of source update, red-black response-matrix sweep and flux
 * reconstruction. For AMD Instinct MI355X (gfx950).
 *
 * Nodes are the bricks of a rectilinear grid; node e = (k * ny + j) * nx + i. Inside a
 * node the flux is expanded in products of Legendre polynomials
 * sqrt((2a+1)(2b+1)(2c+1)) P_a(xi) P_b(eta) P_c(zeta) of total degree a + b + c <=
 * volume_order over the node's reference cube, ordered by total degree, then a
 * descending, then b descending (so moment 0 is the node average). On a face normal to
 * one axis the outward net current is expanded in sqrt((2m+1)(2n+1)) P_m(s) P_n(t) of
 * degree m + n <= face_order in the two other axes taken in increasing order (x faces:
 * y, z; y faces: x, z; z faces: x, y), ordered by degree, m descending. Faces of a node
 * are x-, x+, y-, y+, z-, z+; face DoF index = face * (modes per face) + mode. Partial
 * currents are J+- = phi / 4 +- J / 2 per face moment (Marshak); a vacuum side has no
 * incoming partial current, a reflective side returns the outgoing one.
 *
 * Diffusion data per material and group: D = 1 / (3 Sigma_t) and removal
 * Sigma_r = Sigma_t - Sigma_s(g -> g) > 0; the emission moments of group g are
 * chi_g F / k + sum_{g' != g} Sigma_s(g' -> g) phi_g' (+ external), all groups advancing
 * together from the previous iterate.
 *
 * Conventions are those of moc.h. Solver arrays are FP64, row-major, in node order:
 * moments [N][G][Np] (Np = number of volume modes), partial currents [N][G][Nft]
 * (Nft = 6 * face modes).
 */
#ifndef HFEM_H
#define HFEM_H

#include "moc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct moc_hfem_ctx moc_hfem_ctx;

typedef struct {
    int32_t nx, ny, nz;
    const double *x_edges;          /* host [nx + 1], strictly increasing (cm) */
    const double *y_edges;          /* host [ny + 1] */
    const double *z_edges;          /* host [nz + 1] */
    const int32_t *node_material;   /* host [nz][ny][nx], each in [0, n_materials) */
    int32_t bc[6];                  /* x-, x+, y-, y+, z-, z+: MOC_BC_VACUUM / MOC_BC_REFLECTIVE */
} moc_hfem_grid;

typedef struct {
    int32_t volume_order;     /* complete Legendre degree of the node flux, 0..4 */
    int32_t face_order;       /* complete Legendre degree of the face currents, 0..2, <= volume_order */
    int32_t inner_iterations; /* red-black iterations per sweep (<= 0: 2) */
    int32_t max_iter;         /* moc_hfem_solve iteration limit (<= 0: 10000) */
    int32_t device;           /* HIP device ordinal; negative: host-only context (checks and
                                 info only; device calls return MOC_ESTATE) */
    int32_t check_every;      /* moc_hfem_solve reads (k, residual) back every this many
                                 iterations (<= 0: 1) */
    int32_t fp32_matrices;    /* 0: R and A^-1 stored in FP64 (default); 1: stored in FP32 (half
                                 the bytes of the bandwidth-bound sweep; products, currents,
                                 moments and norms stay FP64) */
} moc_hfem_options;

typedef struct {
    int32_t n_nodes, n_groups;
    int32_t n_moments;        /* Np: volume modes per node and group */
    int32_t n_face_dofs;      /* Nft: face DoFs per node and group (6 faces) */
    int32_t n_red, n_black;   /* nodes of each colour ((i + j + k) even: red) */
    int32_t inner_iterations;
    int64_t device_bytes;
    double setup_ms;          /* host checks, uploads and device preassembly */
    double assemble_ms;       /* device preassembly alone: matrix construction and the two
                                 batched Gauss-Jordan inversions per node and group */
    int32_t fp32_matrices;    /* as in the options */
} moc_hfem_info;

/* Create a context and preassemble, per node and group, the response matrix R of
 * Eq. HFEM_flux_response (J+ = R J- + B s, s_i = (u_i, Q); B s is formed from A^-1 s, as
 * h - R h with h = Lambda^-1 M A^-1 s / 4, so B is not stored) and the inverse reaction
 * matrix A^-1, both computed in FP64. All host arrays are borrowed and copied. Errors:
 * MOC_EINVAL (null pointer, bad sizes or orders, edges not increasing, material out of
 * range, bc not 0/1, Sigma_t <= 0 or Sigma_r <= 0, non-finite data), MOC_ENOMEM, MOC_EHIP. */
int moc_hfem_create(const moc_hfem_grid *grid, const moc_xs *xs, const moc_hfem_options *opts, moc_hfem_ctx **out);
void moc_hfem_destroy(moc_hfem_ctx *ctx);

/* One HFEM solve for given emission moments source_dev (device [N][G][Np], per unit
 * volume): inner_iterations red-black sweeps from the context's partial currents (state
 * carried between calls), then the reconstruction phi = A^-1 (s - M^T (J+ - J-)) into
 * phi_out_dev (device [N][G][Np]). Asynchronous on stream (NULL: the context's). Errors:
 * MOC_EINVAL (null pointer), MOC_ESTATE (host-only), MOC_EHIP. */
int moc_hfem_sweep(moc_hfem_ctx *ctx, const double *source_dev, double *phi_out_dev, void *stream);

/* Power iteration (or source iteration with an external source) from a cold start
 * (phi_0 = 1, higher moments and currents 0, k = 1): each iteration forms the emission
 * moments from the previous iterate, runs one sweep and updates
 * k <- k sum V nuSigma_f phi_0 (new) / sum V nuSigma_f phi_0 (old). Residual: relative
 * V-weighted L2 change of the normalised fission-rate shape (eigen) or of phi_0 (fixed
 * source). Stops when residual and |dk| are both below tol. Synchronous. Errors:
 * MOC_EINVAL (tol <= 0, null out), MOC_ENOCONV (max_iter reached; out still filled in). */
int moc_hfem_solve(moc_hfem_ctx *ctx, double tol, moc_result *out);
/* Exactly n iterations of the same loop from a cold start. */
int moc_hfem_run_iterations(moc_hfem_ctx *ctx, int32_t n, moc_result *out);

/* Flux moments of the last iteration (device [N][G][Np]). */
int moc_hfem_get_flux(moc_hfem_ctx *ctx, double *phi_dev, void *stream);
/* Outgoing partial-current moments (device [N][G][Nft]). */
int moc_hfem_get_currents(moc_hfem_ctx *ctx, double *jplus_dev, void *stream);

/* External source moments (device [N][G][Np], per unit volume, copied), or NULL for the
 * eigenvalue problem. */
int moc_hfem_set_external_source(moc_hfem_ctx *ctx, const double *q_dev);

int moc_hfem_get_info(const moc_hfem_ctx *ctx, moc_hfem_info *info);

/* Device time of the red-black sweeps from HIP events (moc_profile.sweeps counts
 * red-black iterations; sweep_ms is their total). */
int moc_hfem_set_profiling(moc_hfem_ctx *ctx, int32_t enable);
int moc_hfem_get_profile(moc_hfem_ctx *ctx, moc_profile *out);

const char *moc_hfem_last_error(const moc_hfem_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HFEM_H */
