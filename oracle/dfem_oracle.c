/*
 * dfem_oracle.c -- plain FP64 CPU reference for DFEM-SN on 2D triangular meshes.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the HIP DFEM-SN path is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no code, header, table or constant with the product library.
 *
 * What it follows (paper: "Verification and Performance Assessment of NuDEAL"):
 *   - Sec. 2.2, Eq. DFEM_basis: in every element the angular flux and the source of each
 *     discrete ordinate are expansions in N_p local basis functions; here the linear
 *     modal set u_0 = 1, u_1 = (x - x_c) / L, u_2 = (y - y_c) / L on each triangle
 *     (centroid x_c, y_c; L = sqrt(area)), N_p = 3;
 *   - Eq. DFEM_weak / DFEM_parts: test with u_j, integrate by parts:
 *       -int (Omega . grad u_j) psi + int_{boundary} u_j psi* (Omega . n) + Sigma_t int u_j psi
 *         = int u_j q;
 *   - Eq. DFEM_upwind: psi* on a face is the upwind side's trace (the element's own on
 *     outflow faces, the neighbour's on inflow faces);
 *   - discrete ordinates: the angular variable is a set of directions with weights;
 *     scattering is isotropic (Eq. MGNTE's isotropic part).
 *
 * Readings (the paper leaves them open; the same readings are used by the HIP path):
 *   - the problem is planar (no z dependence): each in-plane direction
 *     (sin(theta) cos(phi), sin(theta) sin(phi)) stands for the pair +-mu of polar
 *     cosines and carries both weights; the direction set is passed in;
 *   - vacuum sides give zero inflow; a reflective side gives, for direction m, the
 *     element's own solution for the mirrored direction from the previous sweep (lagged
 *     by one sweep; the fixed point does not depend on the lag);
 *   - scalar-flux moments phi_i = sum_m w_m psi_{m,i}; the emission moments use the same
 *     scattering and fission operators as the flat-source solver, moment by moment;
 *   - the power iteration normalises sum_e area_e nuSigma_f phi_0 = 1 and measures the
 *     residual in the L2 norm of the linear field (phi^T M phi per element and group).
 *
 * Integrals are exact: element mass matrices by the edge-midpoint rule (exact for
 * quadratics on triangles), face integrals by Simpson's rule (exact for quadratics on a
 * segment). Local 3x3 systems are solved by Gaussian elimination with partial pivoting;
 * each direction is swept in a topological order of its upwind dependencies.
 * Parity status of each function is stated in its comment ("pinned by ...").
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define DFO_PI 3.14159265358979323846

typedef struct {
    int nv, nt, M, G, nd;
    double *xy;          /* [nv][2] */
    int *tri;            /* [nt][3] CCW */
    int *mat;            /* [nt] material of each triangle */
    double box[4];
    int bc[4];           /* x = x0, x = x1, y = y0, y = y1: 0 vacuum, 1 reflective */
    double *sigt, *sigs, *nsf, *chi;
    double *mux, *muy, *w;   /* [nd] */
    int *rx, *ry;        /* [nd] mirrored direction across an x side / a y side */
    /* geometry */
    double *area, *cx, *cy, *L;      /* [nt] */
    int *nbr;            /* [nt][3] neighbour across edge k (vertices k, k+1), or -1 - side */
    double *nx, *ny, *len;           /* [nt][3] outward unit normal and length of edge k */
    double *Mm;          /* [nt][3][3] mass matrix */
    double *E;           /* [nt][3][3][3] own face matrices int_f u_j u_i */
    double *C;           /* [nt][3][3][3] coupling int_f u_j (own) u_k (neighbour) */
    /* state */
    double *psi;         /* [nd][nt][G][3] angular flux of the last sweep */
    double *psi_prev;    /* the sweep before (reflective inflow) */
    double *qext;        /* optional external source moments [nt][G][3] */
    int *order;          /* [nd][nt] topological order per direction */
    int *level;          /* [nd][nt] sweep level */
    int max_level;
} dfo_t;

static void *xmalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "dfem oracle: out of memory (%zu bytes)\n", n); abort(); }
    return p;
}

static void basis(const dfo_t *o, int e, double x, double y, double *u) {
    u[0] = 1.0;
    u[1] = (x - o->cx[e]) / o->L[e];
    u[2] = (y - o->cy[e]) / o->L[e];
}

typedef struct { int a, b, t, k; } edge_t;
static int cmp_edge(const void *p, const void *q) {
    const edge_t *x = p, *y = q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    return (x->b > y->b) - (x->b < y->b);
}

/* Which box side an edge lies on (both ends on it), or -1. */
static int side_of_edge(const dfo_t *o, int va, int vb) {
    double tol = 1e-9 * ((o->box[2] - o->box[0]) + (o->box[3] - o->box[1]));
    const double *a = o->xy + 2 * va, *b = o->xy + 2 * vb;
    if (fabs(a[0] - o->box[0]) < tol && fabs(b[0] - o->box[0]) < tol) return 0;
    if (fabs(a[0] - o->box[2]) < tol && fabs(b[0] - o->box[2]) < tol) return 1;
    if (fabs(a[1] - o->box[1]) < tol && fabs(b[1] - o->box[1]) < tol) return 2;
    if (fabs(a[1] - o->box[3]) < tol && fabs(b[1] - o->box[3]) < tol) return 3;
    return -1;
}

/* Topological order and levels of the elements for one direction (Kahn): an element
 * depends on the neighbour across each face with Omega . n < 0. */
static void order_direction(dfo_t *o, int d) {
    int nt = o->nt;
    int *indeg = xmalloc(sizeof(int) * nt), *q = o->order + (size_t)d * nt, *lev = o->level + (size_t)d * nt;
    for (int e = 0; e < nt; e++)
        for (int k = 0; k < 3; k++) {
            double on = o->mux[d] * o->nx[3 * e + k] + o->muy[d] * o->ny[3 * e + k];
            if (on < 0 && o->nbr[3 * e + k] >= 0) indeg[e]++;
        }
    int head = 0, tail = 0;
    for (int e = 0; e < nt; e++) { lev[e] = 0; if (indeg[e] == 0) q[tail++] = e; }
    while (head < tail) {
        int e = q[head++];
        for (int k = 0; k < 3; k++) {
            double on = o->mux[d] * o->nx[3 * e + k] + o->muy[d] * o->ny[3 * e + k];
            int nb = o->nbr[3 * e + k];
            if (on > 0 && nb >= 0) {
                if (lev[nb] < lev[e] + 1) lev[nb] = lev[e] + 1;
                if (--indeg[nb] == 0) q[tail++] = nb;
            }
        }
    }
    if (tail != nt) { fprintf(stderr, "dfem oracle: cyclic sweep dependencies\n"); abort(); }
    for (int e = 0; e < nt; e++) if (lev[e] > o->max_level) o->max_level = lev[e];
    free(indeg);
}

dfo_t *dfo_create(int nv, const double *xy, int nt, const int *tri, const int *tri_region, const int *region_material,
                  const double *box, const int *bc, int M, int G, const double *sigt, const double *sigs,
                  const double *nsf, const double *chi, int nd, const double *mux, const double *muy,
                  const double *w, const int *rx, const int *ry) {
    dfo_t *o = xmalloc(sizeof(dfo_t));
    o->nv = nv; o->nt = nt; o->M = M; o->G = G; o->nd = nd;
    o->xy = xmalloc(sizeof(double) * 2 * nv); memcpy(o->xy, xy, sizeof(double) * 2 * nv);
    o->tri = xmalloc(sizeof(int) * 3 * nt); memcpy(o->tri, tri, sizeof(int) * 3 * nt);
    o->mat = xmalloc(sizeof(int) * nt);
    for (int t = 0; t < nt; t++) o->mat[t] = region_material[tri_region[t]];
    memcpy(o->box, box, sizeof(double) * 4); memcpy(o->bc, bc, sizeof(int) * 4);
    o->sigt = xmalloc(sizeof(double) * M * G); memcpy(o->sigt, sigt, sizeof(double) * M * G);
    o->sigs = xmalloc(sizeof(double) * M * G * G); memcpy(o->sigs, sigs, sizeof(double) * M * G * G);
    o->nsf = xmalloc(sizeof(double) * M * G); memcpy(o->nsf, nsf, sizeof(double) * M * G);
    o->chi = xmalloc(sizeof(double) * M * G); memcpy(o->chi, chi, sizeof(double) * M * G);
    o->mux = xmalloc(sizeof(double) * nd); memcpy(o->mux, mux, sizeof(double) * nd);
    o->muy = xmalloc(sizeof(double) * nd); memcpy(o->muy, muy, sizeof(double) * nd);
    o->w = xmalloc(sizeof(double) * nd); memcpy(o->w, w, sizeof(double) * nd);
    o->rx = xmalloc(sizeof(int) * nd); memcpy(o->rx, rx, sizeof(int) * nd);
    o->ry = xmalloc(sizeof(int) * nd); memcpy(o->ry, ry, sizeof(int) * nd);
    /* element geometry */
    o->area = xmalloc(sizeof(double) * nt); o->cx = xmalloc(sizeof(double) * nt);
    o->cy = xmalloc(sizeof(double) * nt); o->L = xmalloc(sizeof(double) * nt);
    o->nx = xmalloc(sizeof(double) * 3 * nt); o->ny = xmalloc(sizeof(double) * 3 * nt);
    o->len = xmalloc(sizeof(double) * 3 * nt);
    for (int e = 0; e < nt; e++) {
        const double *p0 = xy + 2 * tri[3 * e], *p1 = xy + 2 * tri[3 * e + 1], *p2 = xy + 2 * tri[3 * e + 2];
        o->area[e] = 0.5 * ((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
        o->cx[e] = (p0[0] + p1[0] + p2[0]) / 3.0;
        o->cy[e] = (p0[1] + p1[1] + p2[1]) / 3.0;
        o->L[e] = sqrt(o->area[e]);
        for (int k = 0; k < 3; k++) {
            const double *a = xy + 2 * tri[3 * e + k], *b = xy + 2 * tri[3 * e + (k + 1) % 3];
            double tx = b[0] - a[0], ty = b[1] - a[1], l = sqrt(tx * tx + ty * ty);
            o->len[3 * e + k] = l;
            o->nx[3 * e + k] = ty / l;      /* CCW: outward normal is the tangent turned clockwise */
            o->ny[3 * e + k] = -tx / l;
        }
    }
    /* adjacency by sorting edges */
    edge_t *ed = xmalloc(sizeof(edge_t) * 3 * nt);
    for (int e = 0; e < nt; e++)
        for (int k = 0; k < 3; k++) {
            int a = tri[3 * e + k], b = tri[3 * e + (k + 1) % 3];
            ed[3 * e + k].a = a < b ? a : b; ed[3 * e + k].b = a < b ? b : a;
            ed[3 * e + k].t = e; ed[3 * e + k].k = k;
        }
    qsort(ed, 3 * (size_t)nt, sizeof(edge_t), cmp_edge);
    o->nbr = xmalloc(sizeof(int) * 3 * nt);
    for (int i = 0; i < 3 * nt; i++) o->nbr[i] = -100;
    for (int i = 0; i < 3 * nt; i++) {
        if (i + 1 < 3 * nt && ed[i].a == ed[i + 1].a && ed[i].b == ed[i + 1].b) {
            o->nbr[3 * ed[i].t + ed[i].k] = ed[i + 1].t;
            o->nbr[3 * ed[i + 1].t + ed[i + 1].k] = ed[i].t;
            i++;
        } else {
            int s = side_of_edge(o, ed[i].a, ed[i].b);
            if (s < 0) { fprintf(stderr, "dfem oracle: boundary edge off the box\n"); abort(); }
            o->nbr[3 * ed[i].t + ed[i].k] = -1 - s;
        }
    }
    free(ed);
    /* element and face matrices */
    o->Mm = xmalloc(sizeof(double) * 9 * nt);
    o->E = xmalloc(sizeof(double) * 27 * nt);
    o->C = xmalloc(sizeof(double) * 27 * nt);
    for (int e = 0; e < nt; e++) {
        const int *v = tri + 3 * e;
        for (int k = 0; k < 3; k++) {
            const double *a = xy + 2 * v[k], *b = xy + 2 * v[(k + 1) % 3];
            double mx = 0.5 * (a[0] + b[0]), my = 0.5 * (a[1] + b[1]), u[3];
            basis(o, e, mx, my, u);
            for (int j = 0; j < 3; j++)
                for (int i = 0; i < 3; i++) o->Mm[9 * e + 3 * j + i] += o->area[e] / 3.0 * u[j] * u[i];
            /* Simpson on the face: ends and midpoint */
            double ua[3], ub[3], um[3], na[3], nb_[3], nm[3];
            basis(o, e, a[0], a[1], ua); basis(o, e, b[0], b[1], ub); basis(o, e, mx, my, um);
            int nbr = o->nbr[3 * e + k];
            if (nbr >= 0) { basis(o, nbr, a[0], a[1], na); basis(o, nbr, b[0], b[1], nb_); basis(o, nbr, mx, my, nm); }
            double l = o->len[3 * e + k];
            for (int j = 0; j < 3; j++)
                for (int i = 0; i < 3; i++) {
                    o->E[27 * e + 9 * k + 3 * j + i] = l / 6.0 * (ua[j] * ua[i] + 4.0 * um[j] * um[i] + ub[j] * ub[i]);
                    if (nbr >= 0)
                        o->C[27 * e + 9 * k + 3 * j + i] = l / 6.0 * (ua[j] * na[i] + 4.0 * um[j] * nm[i] + ub[j] * nb_[i]);
                }
        }
    }
    o->order = xmalloc(sizeof(int) * (size_t)nd * nt);
    o->level = xmalloc(sizeof(int) * (size_t)nd * nt);
    for (int d = 0; d < nd; d++) order_direction(o, d);
    o->psi = xmalloc(sizeof(double) * (size_t)nd * nt * G * 3);
    o->psi_prev = xmalloc(sizeof(double) * (size_t)nd * nt * G * 3);
    return o;
}

void dfo_destroy(dfo_t *o) {
    if (!o) return;
    free(o->xy); free(o->tri); free(o->mat); free(o->sigt); free(o->sigs); free(o->nsf); free(o->chi);
    free(o->mux); free(o->muy); free(o->w); free(o->rx); free(o->ry);
    free(o->area); free(o->cx); free(o->cy); free(o->L); free(o->nbr); free(o->nx); free(o->ny); free(o->len);
    free(o->Mm); free(o->E); free(o->C); free(o->order); free(o->level); free(o->psi); free(o->psi_prev);
    free(o->qext); free(o);
}

void dfo_info(const dfo_t *o, int *out /* [2] */) { out[0] = o->max_level + 1; out[1] = o->nt; }
void dfo_geometry(const dfo_t *o, double *area, double *mass /* [nt][9] */, int *nbr /* [nt][3] */, int *level /* [nd][nt] */) {
    if (area) memcpy(area, o->area, sizeof(double) * o->nt);
    if (mass) memcpy(mass, o->Mm, sizeof(double) * 9 * o->nt);
    if (nbr) memcpy(nbr, o->nbr, sizeof(int) * 3 * o->nt);
    if (level) memcpy(level, o->level, sizeof(int) * (size_t)o->nd * o->nt);
}
void dfo_get_psi(const dfo_t *o, double *psi) { memcpy(psi, o->psi, sizeof(double) * (size_t)o->nd * o->nt * o->G * 3); }
void dfo_set_external_source(dfo_t *o, const double *q) {
    free(o->qext); o->qext = NULL;
    if (q) {
        o->qext = xmalloc(sizeof(double) * (size_t)o->nt * o->G * 3);
        memcpy(o->qext, q, sizeof(double) * (size_t)o->nt * o->G * 3);
    }
}

/* Solve a 3x3 system by Gaussian elimination with partial pivoting (A is overwritten). */
static void solve3(double *A, double *b, double *x) {
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++) if (fabs(A[3 * r + c]) > fabs(A[3 * piv + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 3; k++) { double t = A[3 * c + k]; A[3 * c + k] = A[3 * piv + k]; A[3 * piv + k] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < 3; r++) {
            double f = A[3 * r + c] / A[3 * c + c];
            for (int k = c; k < 3; k++) A[3 * r + k] -= f * A[3 * c + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 2; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < 3; k++) s -= A[3 * r + k] * x[k];
        x[r] = s / A[3 * r + r];
    }
}

/* The local system of element e, direction d, total cross section st (Eq. DFEM_parts
 * with the upwind flux of Eq. DFEM_upwind): A psi = b with
 *   A_ji = -(Omega . grad u_j) int u_i + sum_{outflow faces} (Omega . n) int_f u_j u_i + st M_ji
 *   b_j  = sum_i M_ji q_i - sum_{inflow faces} (Omega . n) int_f u_j psi_up.
 * inflow(e, k, out3) supplies int_f u_j psi_up for inflow face k. */
typedef void (*inflow_fn)(const dfo_t *o, void *ctx, int e, int k, double *out3);

static void local_solve(const dfo_t *o, int e, int d, double st, const double *q, inflow_fn inflow, void *ctx, double *psi) {
    double A[9], b[3];
    double gx = o->mux[d] / o->L[e], gy = o->muy[d] / o->L[e];
    double og[3] = {0.0, gx, gy};   /* Omega . grad u_j */
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) A[3 * j + i] = st * o->Mm[9 * e + 3 * j + i] - (i == 0 ? og[j] * o->area[e] : 0.0);
    for (int j = 0; j < 3; j++) {
        b[j] = 0.0;
        for (int i = 0; i < 3; i++) b[j] += o->Mm[9 * e + 3 * j + i] * q[i];
    }
    for (int k = 0; k < 3; k++) {
        double on = o->mux[d] * o->nx[3 * e + k] + o->muy[d] * o->ny[3 * e + k];
        if (on > 0) {
            for (int j = 0; j < 3; j++)
                for (int i = 0; i < 3; i++) A[3 * j + i] += on * o->E[27 * e + 9 * k + 3 * j + i];
        } else if (on < 0) {
            double f[3];
            inflow(o, ctx, e, k, f);
            for (int j = 0; j < 3; j++) b[j] -= on * f[j];
        }
    }
    solve3(A, b, psi);
}

typedef struct { int d, g; } sweep_ctx;
static void sweep_inflow(const dfo_t *o, void *vctx, int e, int k, double *f) {
    sweep_ctx *c = vctx;
    int nb = o->nbr[3 * e + k], G = o->G, nt = o->nt;
    f[0] = f[1] = f[2] = 0.0;
    if (nb >= 0) {
        const double *pn = o->psi + (((size_t)c->d * nt + nb) * G + c->g) * 3;
        for (int j = 0; j < 3; j++)
            for (int i = 0; i < 3; i++) f[j] += o->C[27 * e + 9 * k + 3 * j + i] * pn[i];
        return;
    }
    int side = -1 - nb;
    if (!o->bc[side]) return;
    int dm = side < 2 ? o->rx[c->d] : o->ry[c->d];
    const double *pm = o->psi_prev + (((size_t)dm * nt + e) * G + c->g) * 3;
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) f[j] += o->E[27 * e + 9 * k + 3 * j + i] * pm[i];
}

/* One sweep of every direction and group for emission moments src [nt][G][3] (per unit
 * volume over all directions). Returns the scalar-flux moments phi [nt][G][3].
 * Pinned by: exact reproduction of linear solutions (dfo_sweep_linear), per-sweep
 * balance, infinite medium, symmetry. */
void dfo_sweep(dfo_t *o, const double *src, double *phi) {
    int nt = o->nt, G = o->G, nd = o->nd;
    size_t n = (size_t)nd * nt * G * 3;
    memcpy(o->psi_prev, o->psi, sizeof(double) * n);
    memset(phi, 0, sizeof(double) * (size_t)nt * G * 3);
    for (int d = 0; d < nd; d++)
        for (int g = 0; g < G; g++) {
            sweep_ctx c = {d, g};
            for (int s = 0; s < nt; s++) {
                int e = o->order[(size_t)d * nt + s];
                double q[3];
                for (int i = 0; i < 3; i++) q[i] = src[((size_t)e * G + g) * 3 + i] / (4.0 * DFO_PI);
                double *ps = o->psi + (((size_t)d * nt + e) * G + g) * 3;
                local_solve(o, e, d, o->sigt[o->mat[e] * G + g], q, sweep_inflow, &c, ps);
                for (int i = 0; i < 3; i++) phi[((size_t)e * G + g) * 3 + i] += o->w[d] * ps[i];
            }
        }
}

/* One direction, one group, a per-element linear source q [nt][3] (per steradian,
 * modal) and Sigma_t per element, with every boundary inflow taken from the linear
 * function a + b x + c y: returns psi [nt][3]. Used to pin the discretisation: a linear
 * exact solution is reproduced to round-off. */
typedef struct { double a, b, c; const double *st; double *psi; int d; } lin_ctx;
static void lin_inflow(const dfo_t *o, void *vctx, int e, int k, double *f) {
    lin_ctx *c = vctx;
    int nb = o->nbr[3 * e + k];
    f[0] = f[1] = f[2] = 0.0;
    if (nb >= 0) {
        const double *pn = c->psi + (size_t)nb * 3;
        for (int j = 0; j < 3; j++)
            for (int i = 0; i < 3; i++) f[j] += o->C[27 * e + 9 * k + 3 * j + i] * pn[i];
        return;
    }
    /* Simpson with the exact inflow */
    const double *a = o->xy + 2 * o->tri[3 * e + k], *b = o->xy + 2 * o->tri[3 * e + (k + 1) % 3];
    double mx = 0.5 * (a[0] + b[0]), my = 0.5 * (a[1] + b[1]), l = o->len[3 * e + k];
    double ua[3], ub[3], um[3];
    basis(o, e, a[0], a[1], ua); basis(o, e, b[0], b[1], ub); basis(o, e, mx, my, um);
    double fa = c->a + c->b * a[0] + c->c * a[1], fb = c->a + c->b * b[0] + c->c * b[1], fm = c->a + c->b * mx + c->c * my;
    for (int j = 0; j < 3; j++) f[j] = l / 6.0 * (ua[j] * fa + 4.0 * um[j] * fm + ub[j] * fb);
}
void dfo_sweep_linear(dfo_t *o, int d, const double *st, const double *q, double a, double b, double c, double *psi) {
    lin_ctx ctx = {a, b, c, st, psi, d};
    for (int s = 0; s < o->nt; s++) {
        int e = o->order[(size_t)d * o->nt + s];
        local_solve(o, e, d, st[e], q + 3 * (size_t)e, lin_inflow, &ctx, psi + 3 * (size_t)e);
    }
}

/* Emission moments: s_i = sum_g' Sigma_s,g'->g phi_i,g' + chi_g F_i / k (+ external). */
void dfo_emission(const dfo_t *o, const double *phi, double keff, double *src) {
    int G = o->G;
    for (int e = 0; e < o->nt; e++) {
        int m = o->mat[e];
        for (int i = 0; i < 3; i++) {
            double F = 0.0;
            for (int gp = 0; gp < G; gp++) F += o->nsf[m * G + gp] * phi[((size_t)e * G + gp) * 3 + i];
            for (int g = 0; g < G; g++) {
                double s = o->chi[m * G + g] * F / keff;
                for (int gp = 0; gp < G; gp++) s += o->sigs[((size_t)m * G + gp) * G + g] * phi[((size_t)e * G + gp) * 3 + i];
                if (o->qext) s += o->qext[((size_t)e * G + g) * 3 + i];
                src[((size_t)e * G + g) * 3 + i] = s;
            }
        }
    }
}

static double fission_sum(const dfo_t *o, const double *phi) {
    double fs = 0.0;
    for (int e = 0; e < o->nt; e++)
        for (int g = 0; g < o->G; g++) fs += o->area[e] * o->nsf[o->mat[e] * o->G + g] * phi[((size_t)e * o->G + g) * 3];
    return fs;
}

/* Power (or source) iteration, as the planar oracle's with the linear field's norms. */
int dfo_solve(dfo_t *o, double tol, int max_iter, double *phi, double *k_io, int *iters, double *res_out, double *dk_out,
              int eigen) {
    int nt = o->nt, G = o->G;
    size_t n = (size_t)nt * G * 3, npsi = (size_t)o->nd * nt * G * 3;
    double *src = xmalloc(sizeof(double) * n), *phin = xmalloc(sizeof(double) * n);
    double k = *k_io;
    if (eigen) {
        double fs = fission_sum(o, phi);
        for (size_t i = 0; i < n; i++) phi[i] /= fs;
        for (size_t i = 0; i < npsi; i++) o->psi[i] /= fs;
    }
    int it, conv = 0;
    double res = 1.0, dk = 1.0;
    for (it = 1; it <= max_iter; it++) {
        dfo_emission(o, phi, k, src);
        dfo_sweep(o, src, phin);
        double knew = k;
        if (eigen) {
            double fs = fission_sum(o, phin);
            knew = k * fs;
            for (size_t i = 0; i < n; i++) phin[i] /= fs;
            for (size_t i = 0; i < npsi; i++) o->psi[i] /= fs;
        }
        double num = 0.0, den = 0.0;
        for (int e = 0; e < nt; e++)
            for (int g = 0; g < G; g++) {
                const double *x = phin + ((size_t)e * G + g) * 3, *y = phi + ((size_t)e * G + g) * 3;
                for (int j = 0; j < 3; j++)
                    for (int i = 0; i < 3; i++) {
                        double mji = o->Mm[9 * e + 3 * j + i];
                        num += (x[j] - y[j]) * mji * (x[i] - y[i]);
                        den += x[j] * mji * x[i];
                    }
            }
        res = sqrt(num / den);
        dk = fabs(knew - k);
        k = knew;
        memcpy(phi, phin, sizeof(double) * n);
        if (res < tol && dk < tol) { conv = 1; break; }
    }
    *k_io = k;
    *iters = conv ? it : max_iter;
    *res_out = res;
    *dk_out = dk;
    free(src); free(phin);
    return conv ? 0 : 1;
}
