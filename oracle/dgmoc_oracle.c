/*
 * dgmoc_oracle.c -- plain FP64 CPU reference for DGMOC: planar MOC extended to axially
 * extruded 3D problems by a discontinuous Galerkin discretisation in z.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the HIP DGMOC path is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no code, header, table or constant with the product library. Its
 * tracks and segments come from the planar oracle (moc_oracle.c), passed in as arrays.
 *
 * What it follows (paper: "Verification and Performance Assessment of NuDEAL"):
 *   - Sec. 2.1.1, Eq. DGMOC_expansion: in each axial element (plane) the angular flux
 *     and the source are expanded in n basis functions of z; here n = 2 (the linear
 *     order the paper uses), the Legendre pair u_0 = 1, u_1 = xi on xi in [-1, 1];
 *   - Eq. DGMOC_weak / DGMOC_weak_up: test with u_q, integrate over the plane, take the
 *     angular flux on the upwind axial face from the neighbouring plane (upwinding);
 *     the result along every 2D segment is a 2x2 linear ODE whose solution is a matrix
 *     exponential (written out below);
 *   - Sec. 3.2, Alg. DGMOC_sweep: for each ward (upward, then downward) and each plane in
 *     sweep order: the driven flux, the ray tracing of the plane, the scalar-flux
 *     restoration and the axial interface source for the next plane.
 *
 * The weak form for mu = cos(theta) > 0 (plane height h, local xi, 2D track length s,
 * psi = psi_0 + psi_1 xi, source q = q_0 + q_1 xi per steradian, psi_f the angular flux
 * entering through the lower face) reads, with kappa = mu / h:
 *   sin(theta) dpsi_0/ds = -Sigma_t psi_0 - kappa (psi_0 + psi_1) + q_0 + kappa psi_f
 *   sin(theta) dpsi_1/ds = -Sigma_t psi_1 - 3 kappa (psi_1 - psi_0) + q_1 - 3 kappa psi_f
 * i.e. sin(theta) Psi' = -A Psi + Q with A = Sigma_t I + kappa K, K = [[1, 1], [-3, 3]],
 * Q = (q_0 + kappa psi_f, q_1 - 3 kappa psi_f). Downward directions use the mirrored
 * coordinate xi' = -xi (P1 components change sign), so one form serves both wards.
 *
 * Readings (the paper leaves these open; the same readings are used by the HIP path):
 *   - the upwind face flux psi_f of a direction is flat over each 2D element: the
 *     track-length-weighted average, over that direction's segments in the element, of
 *     the downstream face value psi_0 + psi_1 of the neighbouring plane;
 *   - per-segment averages are tallied directly into both scalar-flux moments;
 *   - at a reflective axial boundary the face flux of direction (a, sense, p) is the
 *     outgoing face flux of the mirrored direction; the bottom face uses the downward
 *     ward of the previous sweep (the upward ward runs first), the top face the upward
 *     ward of the same sweep;
 *   - radial boundary fluxes are updated Jacobi-style between sweeps, per plane, ward
 *     and moment, through the planar tracks' links (reflection keeps mu and psi_1);
 *   - the power iteration normalises sum V h nuSigma_f phi_0 = 1 and measures the
 *     residual in the L2 norm of the linear flux, weights V h for phi_0 and V h / 3
 *     for phi_1.
 *
 * Everything is plain loops in double precision. The matrix exponential is the textbook
 * scaling-and-squaring Taylor series; the segment average comes from integrating the ODE
 * over the segment (a 2x2 solve). Parity status of each function is stated in its
 * comment ("pinned by ...").
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define DGO_PI 3.14159265358979323846

typedef struct {
    /* tracks (from the planar oracle) */
    int T, NA, P, R, M, G, Nz;
    int *t_angle;
    int64_t *t_off;
    int *s_reg;
    double *s_len;
    int *link;               /* [T][2] -> destination track*2+sense, or -1 (vacuum) */
    double *dlt, *wa;        /* per track angle */
    double *mu, *wp, *sinp;  /* per polar angle (one hemisphere) */
    /* axial description */
    double *dz;              /* [Nz] plane heights, bottom to top */
    int *mat;                /* [Nz][R] material of each 3D element */
    int bc_bot, bc_top;      /* 0 vacuum, 1 reflective */
    /* cross sections [M][G], [M][G][G] (from g' to g) */
    double *sigt, *sigs, *nsf, *chi;
    /* derived */
    double *Va;              /* [NA][R] sum over angle-a segments in r of delta_a l */
    double *V;               /* [R] sum_a w_a Va: the planar track-estimated area */
    /* state */
    double *psi, *psi_next;  /* radial boundary [2 wards][Nz][T][2 senses][P][G][2] */
    double *psi_exit;        /* same layout: outgoing flux at the end of each track-sense */
    double *bot;             /* [NA][2][P][R][G] downward outflow through the bottom face */
    double *qext;            /* optional external source [Nz][R][G][2] */
} dgo_t;

static void *xmalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "dg oracle: out of memory (%zu bytes)\n", n); abort(); }
    return p;
}

static size_t psi_count(const dgo_t *o) { return (size_t)2 * o->Nz * o->T * 2 * o->P * o->G * 2; }
static size_t face_count(const dgo_t *o) { return (size_t)o->NA * 2 * o->P * o->R * o->G; }

dgo_t *dgo_create(int T, const int *t_angle, const int64_t *t_off, const int *s_reg, const double *s_len,
                  const int *link, int NA, const double *dlt, const double *wa, int P, const double *mu,
                  const double *wp, int R, int M, int G, const double *sigt, const double *sigs,
                  const double *nsf, const double *chi, int Nz, const double *dz, const int *mat,
                  int bc_bot, int bc_top) {
    dgo_t *o = xmalloc(sizeof(dgo_t));
    o->T = T; o->NA = NA; o->P = P; o->R = R; o->M = M; o->G = G; o->Nz = Nz;
    int64_t S = t_off[T];
    o->t_angle = xmalloc(sizeof(int) * T); memcpy(o->t_angle, t_angle, sizeof(int) * T);
    o->t_off = xmalloc(sizeof(int64_t) * (T + 1)); memcpy(o->t_off, t_off, sizeof(int64_t) * (T + 1));
    o->s_reg = xmalloc(sizeof(int) * S); memcpy(o->s_reg, s_reg, sizeof(int) * S);
    o->s_len = xmalloc(sizeof(double) * S); memcpy(o->s_len, s_len, sizeof(double) * S);
    o->link = xmalloc(sizeof(int) * 2 * T); memcpy(o->link, link, sizeof(int) * 2 * T);
    o->dlt = xmalloc(sizeof(double) * NA); memcpy(o->dlt, dlt, sizeof(double) * NA);
    o->wa = xmalloc(sizeof(double) * NA); memcpy(o->wa, wa, sizeof(double) * NA);
    o->mu = xmalloc(sizeof(double) * P); memcpy(o->mu, mu, sizeof(double) * P);
    o->wp = xmalloc(sizeof(double) * P); memcpy(o->wp, wp, sizeof(double) * P);
    o->sinp = xmalloc(sizeof(double) * P);
    for (int p = 0; p < P; p++) o->sinp[p] = sqrt(1.0 - mu[p] * mu[p]);
    o->sigt = xmalloc(sizeof(double) * M * G); memcpy(o->sigt, sigt, sizeof(double) * M * G);
    o->sigs = xmalloc(sizeof(double) * M * G * G); memcpy(o->sigs, sigs, sizeof(double) * M * G * G);
    o->nsf = xmalloc(sizeof(double) * M * G); memcpy(o->nsf, nsf, sizeof(double) * M * G);
    o->chi = xmalloc(sizeof(double) * M * G); memcpy(o->chi, chi, sizeof(double) * M * G);
    o->dz = xmalloc(sizeof(double) * Nz); memcpy(o->dz, dz, sizeof(double) * Nz);
    o->mat = xmalloc(sizeof(int) * Nz * R); memcpy(o->mat, mat, sizeof(int) * Nz * R);
    o->bc_bot = bc_bot; o->bc_top = bc_top;
    o->Va = xmalloc(sizeof(double) * NA * R);
    o->V = xmalloc(sizeof(double) * R);
    for (int t = 0; t < T; t++) {
        int a = t_angle[t];
        for (int64_t k = t_off[t]; k < t_off[t + 1]; k++) o->Va[(size_t)a * R + s_reg[k]] += dlt[a] * s_len[k];
    }
    for (int a = 0; a < NA; a++)
        for (int r = 0; r < R; r++) o->V[r] += wa[a] * o->Va[(size_t)a * R + r];
    o->psi = xmalloc(sizeof(double) * psi_count(o));
    o->psi_next = xmalloc(sizeof(double) * psi_count(o));
    o->psi_exit = xmalloc(sizeof(double) * psi_count(o));
    o->bot = xmalloc(sizeof(double) * face_count(o));
    return o;
}

void dgo_destroy(dgo_t *o) {
    if (!o) return;
    free(o->t_angle); free(o->t_off); free(o->s_reg); free(o->s_len); free(o->link);
    free(o->dlt); free(o->wa); free(o->mu); free(o->wp); free(o->sinp);
    free(o->sigt); free(o->sigs); free(o->nsf); free(o->chi); free(o->dz); free(o->mat);
    free(o->Va); free(o->V); free(o->psi); free(o->psi_next); free(o->psi_exit); free(o->bot); free(o->qext);
    free(o);
}

void dgo_volumes(const dgo_t *o, double *V, double *Va) {
    memcpy(V, o->V, sizeof(double) * o->R);
    if (Va) memcpy(Va, o->Va, sizeof(double) * o->NA * o->R);
}
void dgo_get_psi(const dgo_t *o, double *psi) { memcpy(psi, o->psi, sizeof(double) * psi_count(o)); }
void dgo_set_psi(dgo_t *o, const double *psi) { memcpy(o->psi, psi, sizeof(double) * psi_count(o)); }
void dgo_get_exit(const dgo_t *o, double *psi) { memcpy(psi, o->psi_exit, sizeof(double) * psi_count(o)); }
void dgo_get_bottom(const dgo_t *o, double *b) { memcpy(b, o->bot, sizeof(double) * face_count(o)); }
void dgo_set_external_source(dgo_t *o, const double *q) {
    free(o->qext); o->qext = NULL;
    if (q) {
        size_t n = (size_t)o->Nz * o->R * o->G * 2;
        o->qext = xmalloc(sizeof(double) * n);
        memcpy(o->qext, q, sizeof(double) * n);
    }
}

/* ------------------------------------------------------------------------------ */
/* 2x2 helpers, row-major m = [m00, m01, m10, m11].                                */
/* ------------------------------------------------------------------------------ */
static void mul2(const double *a, const double *b, double *c) {
    double r0 = a[0] * b[0] + a[1] * b[2], r1 = a[0] * b[1] + a[1] * b[3];
    double r2 = a[2] * b[0] + a[3] * b[2], r3 = a[2] * b[1] + a[3] * b[3];
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}
static void solve2(const double *m, const double *b, double *x) {
    double det = m[0] * m[3] - m[1] * m[2];
    double x0 = (m[3] * b[0] - m[1] * b[1]) / det, x1 = (m[0] * b[1] - m[2] * b[0]) / det;
    x[0] = x0; x[1] = x1;
}

/* e^B for a 2x2 matrix: halve B until its 1-norm is at most 1/2, sum the Taylor     */
/* series until the terms stop changing the sum, square back. Pinned by: agreement  */
/* with scipy.linalg.expm on random and on DGMOC segment matrices.                  */
void dgo_expm2(const double *B, double *E) {
    double nrm = fmax(fabs(B[0]) + fabs(B[2]), fabs(B[1]) + fabs(B[3]));
    int s = 0;
    while (nrm > 0.5) { nrm *= 0.5; s++; }
    double sc = ldexp(1.0, -s);
    double b[4] = {B[0] * sc, B[1] * sc, B[2] * sc, B[3] * sc};
    double term[4] = {1, 0, 0, 1};
    E[0] = 1; E[1] = 0; E[2] = 0; E[3] = 1;
    for (int k = 1; k < 40; k++) {
        mul2(term, b, term);
        for (int i = 0; i < 4; i++) term[i] /= k;
        double tn = fabs(term[0]) + fabs(term[1]) + fabs(term[2]) + fabs(term[3]);
        for (int i = 0; i < 4; i++) E[i] += term[i];
        if (tn < 1e-18) break;
    }
    for (int i = 0; i < s; i++) mul2(E, E, E);
}

/* One segment of the 2x2 characteristic ODE (Eq. DGMOC_weak_up along a segment):   */
/* with f = l / sin(theta), M = f A and Rv = f Q, the ODE over the segment in units  */
/* of its length is Psi' = -M Psi + Rv, so                                          */
/*   Psi_out = e^-M Psi_in + M^-1 (I - e^-M) Rv                                      */
/* and, integrating it once over the segment, the average                           */
/*   Psi_bar = M^-1 (Rv + Psi_in - Psi_out).                                         */
/* Pinned by: the ODE integrated numerically (scipy) on random segments.             */
void dgo_segment(double st, double kap, double f, double q0, double q1, double pf, const double *psi_in,
                 double *psi_out, double *psi_bar) {
    double M[4] = {f * (st + kap), f * kap, -3.0 * f * kap, f * (st + 3.0 * kap)};
    double Rv[2] = {f * (q0 + kap * pf), f * (q1 - 3.0 * kap * pf)};
    double mM[4] = {-M[0], -M[1], -M[2], -M[3]}, E[4];
    dgo_expm2(mM, E);
    double ImE[4] = {1.0 - E[0], -E[1], -E[2], 1.0 - E[3]};
    double w[2] = {ImE[0] * Rv[0] + ImE[1] * Rv[1], ImE[2] * Rv[0] + ImE[3] * Rv[1]}, part[2];
    solve2(M, w, part);
    double out0 = E[0] * psi_in[0] + E[1] * psi_in[1] + part[0];
    double out1 = E[2] * psi_in[0] + E[3] * psi_in[1] + part[1];
    double rhs[2] = {Rv[0] + psi_in[0] - out0, Rv[1] + psi_in[1] - out1};
    solve2(M, rhs, psi_bar);
    psi_out[0] = out0; psi_out[1] = out1;
}

/* ------------------------------------------------------------------------------ */
/* One transport sweep (Alg. DGMOC_sweep with one angle block holding every angle)  */
/* for given emission-density moments src [Nz][R][G][2] (per unit volume, all       */
/* directions; moment 1 is the xi coefficient). Returns phi [Nz][R][G][2] and, if   */
/* asked, the per-plane tallies. Radial boundary fluxes and the bottom-face buffer  */
/* are read from and written back to the oracle's state.                            */
/* Direction weights: 4 pi (w_a / 2)(w_p / 2) per (angle, sense, polar, ward), so   */
/* that all directions sum to 4 pi; a segment contributes weight * delta_a * l *    */
/* Psi_bar to the element's scalar-flux moments, divided by the element's planar    */
/* track-estimated area V_r at the end.                                             */
/* Pinned by: per-sweep neutron balance, the radially infinite slab against an       */
/* independent 1D DG solver, the planar limit (kappa -> 0) against the planar oracle, */
/* the infinite medium, mirror symmetry.                                             */
/* ------------------------------------------------------------------------------ */
void dgo_sweep(dgo_t *o, const double *src, double *phi_out, double *face_flow /* [2][G] or NULL */) {
    int R = o->R, G = o->G, P = o->P, NA = o->NA, Nz = o->Nz, T = o->T;
    size_t nf = face_count(o), ntal = (size_t)Nz * R * G * 2;
    double *tal = xmalloc(sizeof(double) * ntal);
    double *face = xmalloc(sizeof(double) * nf), *next = xmalloc(sizeof(double) * nf);
    if (face_flow) memset(face_flow, 0, sizeof(double) * 2 * G);
    for (int w = 0; w < 2; w++) {
        double sgn = w == 0 ? 1.0 : -1.0;
        /* face flux entering the first plane of this ward */
        if (w == 0) {
            if (o->bc_bot) memcpy(face, o->bot, sizeof(double) * nf);
            else memset(face, 0, sizeof(double) * nf);
        } else if (!o->bc_top) {
            memset(face, 0, sizeof(double) * nf);
        } /* else: face still holds the upward ward's outflow through the top */
        for (int n = 0; n < Nz; n++) {
            int iz = w == 0 ? n : Nz - 1 - n;
            double h = o->dz[iz];
            if (face_flow && n == 0) {
                /* axial inflow through the domain face: sum of weight mu Va psi_f */
                for (int a = 0; a < NA; a++)
                    for (int s = 0; s < 2; s++)
                        for (int p = 0; p < P; p++)
                            for (int r = 0; r < R; r++)
                                for (int g = 0; g < G; g++)
                                    face_flow[g] += DGO_PI * o->wa[a] * o->wp[p] * o->mu[p] * o->Va[(size_t)a * R + r] *
                                                    face[((((size_t)a * 2 + s) * P + p) * R + r) * G + g];
            }
            memset(next, 0, sizeof(double) * nf);
            for (int t = 0; t < T; t++) {
                int a = o->t_angle[t];
                int64_t ns = o->t_off[t + 1] - o->t_off[t];
                for (int s = 0; s < 2; s++)
                    for (int p = 0; p < P; p++) {
                        double kap = o->mu[p] / h, wdir = DGO_PI * o->wa[a] * o->wp[p] * o->dlt[a];
                        for (int g = 0; g < G; g++) {
                            size_t pidx = ((((((size_t)w * Nz + iz) * T + t) * 2 + s) * P + p) * G + g) * 2;
                            double ps[2] = {o->psi[pidx], o->psi[pidx + 1]};
                            for (int64_t i = 0; i < ns; i++) {
                                int64_t k = s ? o->t_off[t + 1] - 1 - i : o->t_off[t] + i;
                                int r = o->s_reg[k], m = o->mat[(size_t)iz * R + r];
                                double l = o->s_len[k];
                                size_t e = (((size_t)iz * R + r) * G + g) * 2;
                                double q0 = src[e] / (4.0 * DGO_PI), q1 = sgn * src[e + 1] / (4.0 * DGO_PI);
                                size_t fi = ((((size_t)a * 2 + s) * P + p) * R + r) * G + g;
                                double out[2], bar[2];
                                dgo_segment(o->sigt[m * G + g], kap, l / o->sinp[p], q0, q1, face[fi], ps, out, bar);
                                tal[e] += wdir * l * bar[0];
                                tal[e + 1] += wdir * l * sgn * bar[1];
                                next[fi] += o->dlt[a] * l * (bar[0] + bar[1]);
                                ps[0] = out[0]; ps[1] = out[1];
                            }
                            o->psi_exit[pidx] = ps[0];
                            o->psi_exit[pidx + 1] = ps[1];
                            int dst = o->link[2 * t + s];
                            if (dst >= 0) {
                                size_t j = ((((((size_t)w * Nz + iz) * T + dst / 2) * 2 + dst % 2) * P + p) * G + g) * 2;
                                o->psi_next[j] = ps[0];
                                o->psi_next[j + 1] = ps[1];
                            }
                        }
                    }
            }
            /* axial interface source for the next plane: flat per element */
            for (int a = 0; a < NA; a++)
                for (int s = 0; s < 2; s++)
                    for (int p = 0; p < P; p++)
                        for (int r = 0; r < R; r++) {
                            double va = o->Va[(size_t)a * R + r];
                            for (int g = 0; g < G; g++) {
                                size_t fi = ((((size_t)a * 2 + s) * P + p) * R + r) * G + g;
                                face[fi] = va > 0 ? next[fi] / va : 0.0;
                            }
                        }
            if (face_flow && n == Nz - 1) {
                for (int a = 0; a < NA; a++)
                    for (int s = 0; s < 2; s++)
                        for (int p = 0; p < P; p++)
                            for (int r = 0; r < R; r++)
                                for (int g = 0; g < G; g++)
                                    face_flow[G + g] += DGO_PI * o->wa[a] * o->wp[p] * o->mu[p] * o->Va[(size_t)a * R + r] *
                                                        face[((((size_t)a * 2 + s) * P + p) * R + r) * G + g];
            }
        }
        if (w == 1) memcpy(o->bot, face, sizeof(double) * nf);
    }
    for (int iz = 0; iz < Nz; iz++)
        for (int r = 0; r < R; r++)
            for (int g = 0; g < G; g++)
                for (int kk = 0; kk < 2; kk++) {
                    size_t e = (((size_t)iz * R + r) * G + g) * 2 + kk;
                    phi_out[e] = tal[e] / o->V[r];
                }
    /* Jacobi: the next sweep enters with this sweep's outgoing fluxes; unlinked      */
    /* (vacuum) entries are zero                                                      */
    double *tmp = o->psi; o->psi = o->psi_next; o->psi_next = tmp;
    memset(o->psi_next, 0, sizeof(double) * psi_count(o));
    free(tal); free(face); free(next);
}

/* Emission-density moments (Eq. MGNTE, isotropic scattering): for k = 0, 1          */
/*   s_k = sum_g' Sigma_s,g'->g phi_k,g' + chi_g F_k / keff (+ external source)       */
/* with F_k = sum_g nuSigma_f,g phi_k,g; the basis is linear, so each moment of the   */
/* emission is the same combination of the flux's moments.                          */
void dgo_emission(const dgo_t *o, const double *phi, double keff, double *src) {
    int R = o->R, G = o->G;
    for (int iz = 0; iz < o->Nz; iz++)
        for (int r = 0; r < R; r++) {
            int m = o->mat[(size_t)iz * R + r];
            const double *ph = phi + ((size_t)iz * R + r) * G * 2;
            for (int kk = 0; kk < 2; kk++) {
                double F = 0.0;
                for (int gp = 0; gp < G; gp++) F += o->nsf[m * G + gp] * ph[gp * 2 + kk];
                for (int g = 0; g < G; g++) {
                    double s = o->chi[m * G + g] * F / keff;
                    for (int gp = 0; gp < G; gp++) s += o->sigs[((size_t)m * G + gp) * G + g] * ph[gp * 2 + kk];
                    if (o->qext) s += o->qext[(((size_t)iz * R + r) * G + g) * 2 + kk];
                    src[(((size_t)iz * R + r) * G + g) * 2 + kk] = s;
                }
            }
        }
}

static double fission_sum(const dgo_t *o, const double *phi) {
    int R = o->R, G = o->G;
    double fs = 0.0;
    for (int iz = 0; iz < o->Nz; iz++)
        for (int r = 0; r < R; r++) {
            int m = o->mat[(size_t)iz * R + r];
            for (int g = 0; g < G; g++)
                fs += o->V[r] * o->dz[iz] * o->nsf[m * G + g] * phi[(((size_t)iz * R + r) * G + g) * 2];
        }
    return fs;
}

static void scale_state(dgo_t *o, double f) {
    size_t np = psi_count(o), nf = face_count(o);
    for (size_t i = 0; i < np; i++) o->psi[i] *= f;
    for (size_t i = 0; i < nf; i++) o->bot[i] *= f;
}

/* Power iteration (eigen) or source iteration (external source, k = 1). Starts from */
/* phi (in/out, [Nz][R][G][2]) and k; every iteration sweeps once with the previous   */
/* iterate's emission, updates k <- k sum V h nuSigma_f phi_0 (new) / (old = 1),       */
/* normalises, and stops when the residual and |dk| are both below tol.               */
int dgo_solve(dgo_t *o, double tol, int max_iter, double *phi, double *k_io, int *iters, double *resid_out,
              double *dk_out, int eigen) {
    int R = o->R, G = o->G, Nz = o->Nz;
    size_t n = (size_t)Nz * R * G * 2;
    double *src = xmalloc(sizeof(double) * n), *phin = xmalloc(sizeof(double) * n);
    double k = *k_io;
    if (eigen) {
        double fs = fission_sum(o, phi);
        for (size_t i = 0; i < n; i++) phi[i] /= fs;
        scale_state(o, 1.0 / fs);
    }
    int it, conv = 0;
    double res = 1.0, dk = 1.0;
    for (it = 1; it <= max_iter; it++) {
        dgo_emission(o, phi, k, src);
        dgo_sweep(o, src, phin, NULL);
        double knew = k;
        if (eigen) {
            double fs = fission_sum(o, phin);
            knew = k * fs;
            for (size_t i = 0; i < n; i++) phin[i] /= fs;
            scale_state(o, 1.0 / fs);
        }
        double num = 0.0, den = 0.0;
        for (int iz = 0; iz < Nz; iz++)
            for (int r = 0; r < R; r++)
                for (int g = 0; g < G; g++)
                    for (int kk = 0; kk < 2; kk++) {
                        size_t e = (((size_t)iz * R + r) * G + g) * 2 + kk;
                        double wgt = o->V[r] * o->dz[iz] * (kk ? 1.0 / 3.0 : 1.0);
                        double d = phin[e] - phi[e];
                        num += wgt * d * d;
                        den += wgt * phin[e] * phin[e];
                    }
        res = sqrt(num / den);
        dk = fabs(knew - k);
        k = knew;
        memcpy(phi, phin, sizeof(double) * n);
        if (res < tol && dk < tol) { conv = 1; break; }
    }
    *k_io = k;
    *iters = conv ? it : max_iter;
    *resid_out = res;
    *dk_out = dk;
    free(src); free(phin);
    return conv ? 0 : 1;
}
