/*
 * moc_oracle.c -- plain FP64 CPU reference for flat-source planar MOC.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the HIP path is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no code, header, table or constant with the product library.
 *
 * What it follows (paper: "Verification and Performance Assessment of NuDEAL"):
 *   - the multigroup k-eigenvalue transport equation with isotropic scattering and a
 *     fission source (Sec. 2, Eq. MGNTE and its per-element form, Eq. MGNTE_element);
 *   - flat-source regions = mesh elements (Sec. 2.1);
 *   - the characteristic equation along straight tracks (Eq. MOC_eq) and its segment
 *     solution with exponential attenuation (Eq. MOC_sol);
 *   - scalar flux by angular integration over all discrete directions (Sec. 2.1);
 *   - modular (cyclic) rays laid on the bounding box of the whole domain, and
 *     ray-mesh intersection yielding per-segment (length, element) (Sec. 3.1).
 * The paper leaves the laydown formulas, quadratures, tally form, volumes and the
 * iteration scheme unstated; the readings used here are written next to each step.
 *
 * Everything is plain loops in double precision with libm exp/expm1. Tracking is done
 * by clipping every track line against every triangle whose projection it crosses
 * (a different algorithm from the product library's mesh walk).
 *
 * Parity status of each function is stated in its comment ("pinned by ...").
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

typedef struct {
    /* problem */
    int nv, nt, R, M, G;
    double *xy;
    int *tri, *tri_region, *region_material;
    int domain;            /* 0 box, 1 hexagon */
    double box[4];         /* x0 y0 x1 y1 */
    double hex_apothem;
    int bc[6];
    double *sigt, *sigs, *nsf, *chi; /* [M][G], [M][G][G] from->to, [M][G], [M][G] */
    /* quadrature and laydown */
    int A, P, NA;          /* NA = A/2 track angles in (0, pi) */
    double spacing;
    double *phi, *dlt, *wa; /* per track angle */
    int *nx, *ny;
    double *mu, *wp, *sinp; /* polar, per hemisphere */
    /* tracks */
    int T;
    int *t_angle;
    double *t_x0, *t_y0, *t_x1, *t_y1, *t_len;
    int64_t *t_off;        /* [T+1] into segment arrays */
    int *s_reg;
    double *s_len;
    int64_t S;
    int *link;             /* [T][2] -> destination (track*2+sense) or -1 */
    double *V;             /* track-estimated region volume */
    /* state */
    double *psi;           /* [T][2][P][G] incoming angular flux for each track-sense */
    double *psi_next;
    double *psi_exit;      /* [T][2][P][G] outgoing angular flux of the last sweep */
    double *qext;          /* optional external source [R][G] (emission density) */
    int gs_boundary;       /* 1: boundary Gauss-Seidel inside a sweep */
    int gs_energy;         /* 1: energy Gauss-Seidel inside a power iteration */
    int nthreads;          /* threads of the track loop (1 = serial) */
    double max_gap;        /* largest uncovered gap found while tracking (diagnostic) */
    /* coarse mesh for CMFD (off when n_cells == 0): surface partial currents */
    int n_cells;
    int *region_cell;      /* [R] coarse cell of each region */
    int64_t *nbr_off;      /* [n_cells + 1] neighbour slots of each cell */
    int *nbr;              /* neighbour cell of each slot; -1 = the domain boundary */
    double *jpart;         /* [slots][G] partial current leaving the cell through the slot */
    double *jin_bnd;       /* [n_cells][G] partial current entering the cell from outside */
    char err[256];
} orc_t;

static int g_default_threads = 1;   /* threads of contexts created from now on */
void orc_set_default_threads(int n) { g_default_threads = n > 0 ? n : 1; }

static void *xmalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", n); abort(); }
    return p;
}

/* ------------------------------------------------------------------------------ */
/* Polar quadrature: half-range Gauss-Legendre (reading: the paper names no polar  */
/* set). The positive roots of the Legendre polynomial of degree 2P with their     */
/* weights; the weights of one hemisphere sum to 1. Newton iteration on the three- */
/* term recurrence. Pinned against a library Gauss-Legendre routine and against    */
/* exact moments of mu^k.                                                          */
/* ------------------------------------------------------------------------------ */
int orc_polar_gl(int P, double *mu, double *w) {
    int n = 2 * P;
    for (int i = 0; i < P; i++) {
        /* i-th largest root; initial guess from the Chebyshev-like asymptotic */
        double x = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            /* p1 = P_n(x), p0 = P_{n-1}(x) */
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        mu[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* Cyclic track laydown on the bounding box W x H (reading of the modular-ray      */
/* method on the whole-domain box, Sec. 3.1; formulas are the usual correction so  */
/* that track ends meet on every side):                                            */
/*   phi0_a = 2 pi (a + 1/2) / A,  nx = ceil(W sin phi0 / d), ny = ceil(H cos phi0/d) */
/*   phi_a = atan(H nx / (W ny)),  delta_a = (W / nx) sin phi_a                    */
/* for a < A/4; the angle pi - phi_a reuses nx, ny, delta_a. Azimuthal weights are */
/* the midpoint rule on the sorted angles over [0, pi]. Pinned by: sum of weights  */
/* = 1, total track volume = W*H exactly, delta_a <= d.                            */
/* ------------------------------------------------------------------------------ */
int orc_layout(double W, double H, int A, double d, double *phi, double *dlt, int *nx,
               int *ny, double *wa) {
    if (A <= 0 || A % 4) return -1;
    int NA = A / 2, NQ = A / 4;
    for (int a = 0; a < NQ; a++) {
        double p0 = 2.0 * ORC_PI * (a + 0.5) / A;
        int mx = (int)ceil(W * sin(p0) / d);
        int my = (int)ceil(H * cos(p0) / d);
        double p = atan((H * mx) / (W * my));
        double dl = (W / mx) * sin(p);
        phi[a] = p; dlt[a] = dl; nx[a] = mx; ny[a] = my;
        int b = NA - 1 - a;
        phi[b] = ORC_PI - p; dlt[b] = dl; nx[b] = mx; ny[b] = my;
    }
    for (int a = 0; a < NA; a++) {
        double lo = (a == 0) ? 0.0 : 0.5 * (phi[a - 1] + phi[a]);
        double hi = (a == NA - 1) ? ORC_PI : 0.5 * (phi[a] + phi[a + 1]);
        wa[a] = (hi - lo) / ORC_PI;
    }
    return 0;
}

/* clip the line p + s*u against a convex polygon given by inward half-planes
 * n_i . x >= c_i; returns 0 if empty. */
static int clip_convex(double px, double py, double ux, double uy, int nh, const double *nxs,
                       const double *nys, const double *cs, double *s0, double *s1) {
    double lo = -1e300, hi = 1e300;
    for (int i = 0; i < nh; i++) {
        double den = nxs[i] * ux + nys[i] * uy;
        double num = cs[i] - (nxs[i] * px + nys[i] * py);
        if (den == 0.0) {
            if (num > 0.0) return 0;
            continue;
        }
        double s = num / den;
        if (den > 0) { if (s > lo) lo = s; }
        else { if (s < hi) hi = s; }
    }
    *s0 = lo; *s1 = hi;
    return hi > lo;
}

static void domain_halfplanes(const orc_t *o, int *nh, double *nxs, double *nys, double *cs) {
    if (o->domain == 0) {
        *nh = 4;
        nxs[0] = 1; nys[0] = 0; cs[0] = o->box[0];
        nxs[1] = -1; nys[1] = 0; cs[1] = -o->box[2];
        nxs[2] = 0; nys[2] = 1; cs[2] = o->box[1];
        nxs[3] = 0; nys[3] = -1; cs[3] = -o->box[3];
    } else {
        double cx = 0.5 * (o->box[0] + o->box[2]), cy = 0.5 * (o->box[1] + o->box[3]);
        *nh = 6;
        for (int k = 0; k < 6; k++) {
            double ang = (30.0 + 60.0 * k) * ORC_PI / 180.0;
            /* inward normal = -outward */
            nxs[k] = -cos(ang); nys[k] = -sin(ang);
            cs[k] = nxs[k] * cx + nys[k] * cy - o->hex_apothem;
        }
    }
}

typedef struct { int trk; double s0, s1; int reg; } piece_t;

static int cmp_piece(const void *a, const void *b) {
    const piece_t *x = a, *y = b;
    if (x->trk != y->trk) return x->trk < y->trk ? -1 : 1;
    if (x->s0 != y->s0) return x->s0 < y->s0 ? -1 : 1;
    return 0;
}

typedef struct { double c; int t; } cidx_t;
static int cmp_cidx(const void *a, const void *b) {
    const cidx_t *x = a, *y = b;
    return (x->c > y->c) - (x->c < y->c);
}

/* ------------------------------------------------------------------------------ */
/* Track generation and ray tracing.                                               */
/* Tracks of angle phi start at x = (i + 1/2) W / nx on the bottom side and at     */
/* y = (j + 1/2) H / ny on the left side (right side when phi > pi/2), run in the  */
/* direction (cos phi, sin phi) ("forward" sense) and are clipped to the domain.   */
/* Each track is cut at every triangle it crosses: the piece inside a triangle is  */
/* the clip of the line against the triangle's three half-planes. Pieces are       */
/* ordered along the track; pieces shorter than 1e-12 cm are dropped, then         */
/* consecutive pieces in the same region are merged (exact under a flat source).   */
/* Canonical track order: by angle index, then by the perpendicular coordinate     */
/* n . x with n = (-sin phi, cos phi). Pinned by: every track's piece lengths sum  */
/* to its chord, sum of volumes = W*H, agreement with an independent walker.       */
/* ------------------------------------------------------------------------------ */
/* Segments of the tracks [tfirst, tlast) of angle a: clip every track of the angle   */
/* against every triangle whose projection it crosses, order the pieces along each    */
/* track, drop pieces shorter than 1e-12 cm, then merge consecutive pieces of the same */
/* region. Output: per-track offsets (relative), regions, lengths, the largest gap.    */
typedef struct { int64_t n; int64_t *off; int *reg; double *len; double max_gap; } angle_segs_t;

static void trace_angle(const orc_t *o, int a, int tfirst, int tlast, angle_segs_t *out) {
    int nta = tlast - tfirst;
    double ph = o->phi[a], ux = cos(ph), uy = sin(ph);
    double nxn = -uy, nyn = ux;
    double *c = xmalloc(sizeof(double) * (nta ? nta : 1));
    for (int k = 0; k < nta; k++) c[k] = nxn * o->t_x0[tfirst + k] + nyn * o->t_y0[tfirst + k];
    int64_t cap = 1 << 16, np = 0;
    piece_t *pc = xmalloc(sizeof(piece_t) * cap);
    for (int e = 0; e < o->nt; e++) {
        const int *v = o->tri + 3 * e;
        double px[3], py[3], pmin = 1e300, pmax = -1e300;
        for (int q = 0; q < 3; q++) {
            px[q] = o->xy[2 * v[q]]; py[q] = o->xy[2 * v[q] + 1];
            double pr = nxn * px[q] + nyn * py[q];
            if (pr < pmin) pmin = pr;
            if (pr > pmax) pmax = pr;
        }
        /* triangle half-planes (CCW => inward normal of edge (p,q) is (-(qy-py), qx-px)) */
        double ex[3], ey[3], ec[3];
        for (int q = 0; q < 3; q++) {
            int r = (q + 1) % 3;
            ex[q] = -(py[r] - py[q]); ey[q] = px[r] - px[q];
            ec[q] = ex[q] * px[q] + ey[q] * py[q];
        }
        /* first track with c > pmin */
        int lo = 0, hi = nta;
        while (lo < hi) { int mid = (lo + hi) / 2; if (c[mid] <= pmin) lo = mid + 1; else hi = mid; }
        for (int k = lo; k < nta && c[k] < pmax; k++) {
            int t = tfirst + k;
            double s0, s1;
            if (!clip_convex(o->t_x0[t], o->t_y0[t], ux, uy, 3, ex, ey, ec, &s0, &s1)) continue;
            if (np == cap) { cap *= 2; pc = realloc(pc, sizeof(piece_t) * cap); if (!pc) abort(); }
            pc[np].trk = t; pc[np].s0 = s0; pc[np].s1 = s1; pc[np].reg = o->tri_region[e];
            np++;
        }
    }
    free(c);
    qsort(pc, np, sizeof(piece_t), cmp_piece);
    int64_t scap = np > 0 ? np : 1, S = 0;
    int *sreg = xmalloc(sizeof(int) * scap);
    double *slen = xmalloc(sizeof(double) * scap);
    int64_t *off = xmalloc(sizeof(int64_t) * (nta ? nta : 1));
    double max_gap = 0.0;
    int64_t i = 0;
    for (int t = tfirst; t < tlast; t++) {
        off[t - tfirst] = S;
        double last_end = 0.0;
        int prev = -1;
        for (; i < np && pc[i].trk == t; i++) {
            double L = pc[i].s1 - pc[i].s0;
            if (L < 1e-12) continue;            /* drop first ... */
            double g = pc[i].s0 - last_end;     /* pieces must tile the chord */
            if (fabs(g) > max_gap) max_gap = fabs(g);
            if (pc[i].s1 > last_end) last_end = pc[i].s1;
            if (prev == pc[i].reg) {             /* ... then merge */
                slen[S - 1] += L;
                continue;
            }
            sreg[S] = pc[i].reg; slen[S] = L; S++;
            prev = pc[i].reg;
        }
        double g = o->t_len[t] - last_end;
        if (fabs(g) > max_gap) max_gap = fabs(g);
    }
    free(pc);
    out->n = S; out->off = off; out->reg = sreg; out->len = slen; out->max_gap = max_gap;
}

static int trace(orc_t *o) {
    double W = o->box[2] - o->box[0], H = o->box[3] - o->box[1];
    int NA = o->NA;
    /* count candidate tracks */
    int Tmax = 0;
    for (int a = 0; a < NA; a++) Tmax += o->nx[a] + o->ny[a];
    int nh; double hnx[6], hny[6], hc[6];
    domain_halfplanes(o, &nh, hnx, hny, hc);
    o->t_angle = xmalloc(sizeof(int) * Tmax);
    o->t_x0 = xmalloc(sizeof(double) * Tmax); o->t_y0 = xmalloc(sizeof(double) * Tmax);
    o->t_x1 = xmalloc(sizeof(double) * Tmax); o->t_y1 = xmalloc(sizeof(double) * Tmax);
    o->t_len = xmalloc(sizeof(double) * Tmax);
    int T = 0;
    cidx_t *ci = xmalloc(sizeof(cidx_t) * Tmax);
    for (int a = 0; a < NA; a++) {
        double ph = o->phi[a], ux = cos(ph), uy = sin(ph);
        double nxn = -uy, nyn = ux;
        int n0 = 0;
        for (int i = 0; i < o->nx[a]; i++) {
            double x = o->box[0] + (i + 0.5) * W / o->nx[a], y = o->box[1];
            o->t_x0[T + n0] = x; o->t_y0[T + n0] = y; n0++;
        }
        for (int j = 0; j < o->ny[a]; j++) {
            double x = (ph < 0.5 * ORC_PI) ? o->box[0] : o->box[2];
            double y = o->box[1] + (j + 0.5) * H / o->ny[a];
            o->t_x0[T + n0] = x; o->t_y0[T + n0] = y; n0++;
        }
        /* sort this angle's tracks by perpendicular coordinate */
        for (int k = 0; k < n0; k++) {
            ci[k].c = nxn * o->t_x0[T + k] + nyn * o->t_y0[T + k];
            ci[k].t = k;
        }
        qsort(ci, n0, sizeof(cidx_t), cmp_cidx);
        double *tx = xmalloc(sizeof(double) * n0), *ty = xmalloc(sizeof(double) * n0);
        for (int k = 0; k < n0; k++) { tx[k] = o->t_x0[T + ci[k].t]; ty[k] = o->t_y0[T + ci[k].t]; }
        int kept = 0;
        for (int k = 0; k < n0; k++) {
            double s0, s1;
            if (!clip_convex(tx[k], ty[k], ux, uy, nh, hnx, hny, hc, &s0, &s1)) continue;
            if (s1 - s0 <= 1e-12) continue;
            int t = T + kept;
            o->t_angle[t] = a;
            o->t_x0[t] = tx[k] + s0 * ux; o->t_y0[t] = ty[k] + s0 * uy;
            o->t_x1[t] = tx[k] + s1 * ux; o->t_y1[t] = ty[k] + s1 * uy;
            o->t_len[t] = s1 - s0;
            kept++;
        }
        free(tx); free(ty);
        T += kept;
    }
    free(ci);
    o->T = T;

    /* pieces, angle by angle; the angles are independent, so they may run on several   */
    /* threads (each angle's segments in arrays of its own, joined in angle order after) */
    o->t_off = xmalloc(sizeof(int64_t) * (T + 1));
    o->max_gap = 0.0;
    int *afirst = xmalloc(sizeof(int) * (NA + 1));
    {
        int t = 0;
        for (int a = 0; a < NA; a++) {
            afirst[a] = t;
            while (t < T && o->t_angle[t] == a) t++;
        }
        afirst[NA] = T;
    }
    angle_segs_t *as = xmalloc(sizeof(angle_segs_t) * (NA ? NA : 1));
    int nth = o->nthreads > 0 ? o->nthreads : 1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nth) schedule(dynamic, 1)
#endif
    for (int a = 0; a < NA; a++) trace_angle(o, a, afirst[a], afirst[a + 1], &as[a]);
    int64_t S = 0;
    for (int a = 0; a < NA; a++) S += as[a].n;
    int *sreg = xmalloc(sizeof(int) * (S ? S : 1));
    double *slen = xmalloc(sizeof(double) * (S ? S : 1));
    int64_t pos = 0;
    for (int a = 0; a < NA; a++) {
        for (int t = afirst[a]; t < afirst[a + 1]; t++) o->t_off[t] = pos + as[a].off[t - afirst[a]];
        memcpy(sreg + pos, as[a].reg, sizeof(int) * as[a].n);
        memcpy(slen + pos, as[a].len, sizeof(double) * as[a].n);
        pos += as[a].n;
        if (as[a].max_gap > o->max_gap) o->max_gap = as[a].max_gap;
        free(as[a].off); free(as[a].reg); free(as[a].len);
    }
    o->t_off[T] = S;
    free(as); free(afirst);
    o->s_reg = sreg; o->s_len = slen; o->S = S;
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* Boundary links (reading: reflective sides send the outgoing angular flux of a   */
/* track-sense into the track-sense that starts at the same boundary point in the  */
/* mirrored direction; vacuum sides give zero incoming flux).                      */
/* ------------------------------------------------------------------------------ */
typedef struct { double pos; int ts; double dx, dy; } start_t;
static int cmp_start(const void *a, const void *b) {
    const start_t *x = a, *y = b;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

static int side_of(const orc_t *o, double x, double y, double *pos) {
    double W = o->box[2] - o->box[0], H = o->box[3] - o->box[1];
    double tol = 1e-9 * (W + H);
    if (fabs(x - o->box[0]) < tol) { *pos = y; return 0; }
    if (fabs(x - o->box[2]) < tol) { *pos = y; return 1; }
    if (fabs(y - o->box[1]) < tol) { *pos = x; return 2; }
    if (fabs(y - o->box[3]) < tol) { *pos = x; return 3; }
    return -1;
}

static int make_links(orc_t *o) {
    int T = o->T;
    o->link = xmalloc(sizeof(int) * 2 * T);
    for (int i = 0; i < 2 * T; i++) o->link[i] = -1;
    if (o->domain != 0) return 0; /* hexagon: vacuum only */
    start_t *st[4];
    int ns[4] = {0, 0, 0, 0};
    for (int s = 0; s < 4; s++) st[s] = xmalloc(sizeof(start_t) * 2 * T);
    for (int t = 0; t < T; t++) {
        double ph = o->phi[o->t_angle[t]], ux = cos(ph), uy = sin(ph);
        for (int sense = 0; sense < 2; sense++) {
            double x = sense ? o->t_x1[t] : o->t_x0[t];
            double y = sense ? o->t_y1[t] : o->t_y0[t];
            double pos;
            int sd = side_of(o, x, y, &pos);
            if (sd < 0) { snprintf(o->err, sizeof o->err, "track start off the box"); return -1; }
            start_t *e = &st[sd][ns[sd]++];
            e->pos = pos; e->ts = 2 * t + sense;
            e->dx = sense ? -ux : ux; e->dy = sense ? -uy : uy;
        }
    }
    for (int s = 0; s < 4; s++) qsort(st[s], ns[s], sizeof(start_t), cmp_start);
    double W = o->box[2] - o->box[0], H = o->box[3] - o->box[1];
    double tol = 1e-9 * (W + H);
    for (int t = 0; t < T; t++) {
        double ph = o->phi[o->t_angle[t]], ux = cos(ph), uy = sin(ph);
        for (int sense = 0; sense < 2; sense++) {
            double x = sense ? o->t_x0[t] : o->t_x1[t]; /* exit point */
            double y = sense ? o->t_y0[t] : o->t_y1[t];
            double dx = sense ? -ux : ux, dy = sense ? -uy : uy;
            double pos;
            int sd = side_of(o, x, y, &pos);
            if (sd < 0) { snprintf(o->err, sizeof o->err, "track end off the box"); return -1; }
            if (o->bc[sd] == 0) continue; /* vacuum */
            double rx = (sd < 2) ? -dx : dx, ry = (sd < 2) ? dy : -dy;
            /* find the start record at pos with direction (rx, ry) */
            int lo = 0, hi = ns[sd];
            while (lo < hi) { int mid = (lo + hi) / 2; if (st[sd][mid].pos < pos - tol) lo = mid + 1; else hi = mid; }
            int found = -1;
            for (int k = lo; k < ns[sd] && st[sd][k].pos <= pos + tol; k++) {
                if (st[sd][k].dx * rx + st[sd][k].dy * ry > 1.0 - 1e-9) { found = st[sd][k].ts; break; }
            }
            if (found < 0) { snprintf(o->err, sizeof o->err, "no reflected track at side %d pos %.17g", sd, pos); return -1; }
            o->link[2 * t + sense] = found;
        }
    }
    for (int s = 0; s < 4; s++) free(st[s]);
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* Track-estimated volumes V_r = sum_a w_a delta_a sum_{k in r} l_k (reading: the  */
/* paper gives no volume definition; this is the one that makes the flat-source    */
/* term of the scalar flux exact). Pinned: sum V_r = W*H on box domains.           */
/* ------------------------------------------------------------------------------ */
static void volumes(orc_t *o) {
    o->V = xmalloc(sizeof(double) * o->R);
    for (int t = 0; t < o->T; t++) {
        int a = o->t_angle[t];
        for (int64_t k = o->t_off[t]; k < o->t_off[t + 1]; k++)
            o->V[o->s_reg[k]] += o->wa[a] * o->dlt[a] * o->s_len[k];
    }
}

/* ------------------------------------------------------------------------------ */
/* public: create / destroy / accessors                                            */
/* ------------------------------------------------------------------------------ */
orc_t *orc_create(int nv, const double *xy, int nt, const int *tri, const int *tri_region,
                  int R, const int *region_material, int domain, const double *box,
                  double hex_apothem, const int *bc, int M, int G, const double *sigt,
                  const double *sigs, const double *nsf, const double *chi, int A, int P,
                  double spacing, char *errbuf, int errlen) {
    orc_t *o = xmalloc(sizeof(orc_t));
    o->nv = nv; o->nt = nt; o->R = R; o->M = M; o->G = G;
    o->xy = xmalloc(sizeof(double) * 2 * nv); memcpy(o->xy, xy, sizeof(double) * 2 * nv);
    o->tri = xmalloc(sizeof(int) * 3 * nt); memcpy(o->tri, tri, sizeof(int) * 3 * nt);
    o->tri_region = xmalloc(sizeof(int) * nt); memcpy(o->tri_region, tri_region, sizeof(int) * nt);
    o->region_material = xmalloc(sizeof(int) * R);
    memcpy(o->region_material, region_material, sizeof(int) * R);
    o->domain = domain;
    memcpy(o->box, box, sizeof(double) * 4);
    o->hex_apothem = hex_apothem;
    memcpy(o->bc, bc, sizeof(int) * (domain == 0 ? 4 : 6));
    o->sigt = xmalloc(sizeof(double) * M * G); memcpy(o->sigt, sigt, sizeof(double) * M * G);
    o->sigs = xmalloc(sizeof(double) * M * G * G); memcpy(o->sigs, sigs, sizeof(double) * M * G * G);
    o->nsf = xmalloc(sizeof(double) * M * G); memcpy(o->nsf, nsf, sizeof(double) * M * G);
    o->chi = xmalloc(sizeof(double) * M * G); memcpy(o->chi, chi, sizeof(double) * M * G);
    o->A = A; o->P = P; o->NA = A / 2; o->spacing = spacing;
    o->nthreads = g_default_threads;
    int NA = A / 2;
    o->phi = xmalloc(sizeof(double) * NA); o->dlt = xmalloc(sizeof(double) * NA);
    o->wa = xmalloc(sizeof(double) * NA);
    o->nx = xmalloc(sizeof(int) * NA); o->ny = xmalloc(sizeof(int) * NA);
    if (orc_layout(box[2] - box[0], box[3] - box[1], A, spacing, o->phi, o->dlt, o->nx, o->ny, o->wa)) {
        snprintf(errbuf, errlen, "n_azim must be a positive multiple of 4");
        return NULL;
    }
    o->mu = xmalloc(sizeof(double) * P); o->wp = xmalloc(sizeof(double) * P);
    o->sinp = xmalloc(sizeof(double) * P);
    orc_polar_gl(P, o->mu, o->wp);
    for (int p = 0; p < P; p++) o->sinp[p] = sqrt(1.0 - o->mu[p] * o->mu[p]);
    trace(o);
    if (make_links(o)) { snprintf(errbuf, errlen, "%s", o->err); return NULL; }
    volumes(o);
    o->psi = xmalloc(sizeof(double) * (size_t)o->T * 2 * P * G);
    o->psi_next = xmalloc(sizeof(double) * (size_t)o->T * 2 * P * G);
    o->psi_exit = xmalloc(sizeof(double) * (size_t)o->T * 2 * P * G);
    return o;
}

void orc_destroy(orc_t *o) {
    if (!o) return;
    free(o->xy); free(o->tri); free(o->tri_region); free(o->region_material);
    free(o->sigt); free(o->sigs); free(o->nsf); free(o->chi);
    free(o->phi); free(o->dlt); free(o->wa); free(o->nx); free(o->ny);
    free(o->mu); free(o->wp); free(o->sinp);
    free(o->t_angle); free(o->t_x0); free(o->t_y0); free(o->t_x1); free(o->t_y1); free(o->t_len);
    free(o->t_off); free(o->s_reg); free(o->s_len); free(o->link); free(o->V);
    free(o->psi); free(o->psi_next); free(o->psi_exit); free(o->qext);
    free(o->region_cell); free(o->nbr_off); free(o->nbr); free(o->jpart); free(o->jin_bnd);
    free(o);
}

/* counts: T, S, NA, max_gap */
void orc_info(const orc_t *o, int64_t *out /* [4] */, double *max_gap) {
    out[0] = o->T; out[1] = o->S; out[2] = o->NA; out[3] = o->P;
    *max_gap = o->max_gap;
}
void orc_angles(const orc_t *o, double *phi, double *dlt, double *wa, int *nx, int *ny) {
    memcpy(phi, o->phi, sizeof(double) * o->NA); memcpy(dlt, o->dlt, sizeof(double) * o->NA);
    memcpy(wa, o->wa, sizeof(double) * o->NA);
    memcpy(nx, o->nx, sizeof(int) * o->NA); memcpy(ny, o->ny, sizeof(int) * o->NA);
}
void orc_polar(const orc_t *o, double *mu, double *w) {
    memcpy(mu, o->mu, sizeof(double) * o->P); memcpy(w, o->wp, sizeof(double) * o->P);
}
void orc_tracks(const orc_t *o, int *angle, double *xy01 /* [T][4] */, double *len, int64_t *off,
                int *link) {
    for (int t = 0; t < o->T; t++) {
        angle[t] = o->t_angle[t];
        xy01[4 * t] = o->t_x0[t]; xy01[4 * t + 1] = o->t_y0[t];
        xy01[4 * t + 2] = o->t_x1[t]; xy01[4 * t + 3] = o->t_y1[t];
        len[t] = o->t_len[t];
        link[2 * t] = o->link[2 * t]; link[2 * t + 1] = o->link[2 * t + 1];
    }
    memcpy(off, o->t_off, sizeof(int64_t) * (o->T + 1));
}
void orc_segments(const orc_t *o, int *reg, double *len) {
    memcpy(reg, o->s_reg, sizeof(int) * o->S); memcpy(len, o->s_len, sizeof(double) * o->S);
}
void orc_volumes(const orc_t *o, double *V) { memcpy(V, o->V, sizeof(double) * o->R); }
void orc_get_psi(const orc_t *o, double *psi) {
    memcpy(psi, o->psi, sizeof(double) * (size_t)o->T * 2 * o->P * o->G);
}
void orc_set_psi(orc_t *o, const double *psi) {
    memcpy(o->psi, psi, sizeof(double) * (size_t)o->T * 2 * o->P * o->G);
}
void orc_get_exit_psi(const orc_t *o, double *psi) {
    memcpy(psi, o->psi_exit, sizeof(double) * (size_t)o->T * 2 * o->P * o->G);
}
void orc_set_options(orc_t *o, int gs_boundary, int gs_energy) {
    o->gs_boundary = gs_boundary; o->gs_energy = gs_energy;
}
void orc_set_external_source(orc_t *o, const double *q) {
    free(o->qext); o->qext = NULL;
    if (q) {
        o->qext = xmalloc(sizeof(double) * o->R * o->G);
        memcpy(o->qext, q, sizeof(double) * o->R * o->G);
    }
}

/* ------------------------------------------------------------------------------ */
/* One transport sweep of group g over every track, sense and polar angle, for a   */
/* given flat source qhat[r] = q/Sigma_t (the per-steradian source over Sigma_t).  */
/* Along each segment, Eq. MOC_sol gives psi_out = qhat + (psi_in - qhat) e^-tau   */
/* with tau = Sigma_t l / sin(theta_p) (l is the planar length). The increment     */
/* Delta = psi_in - psi_out is tallied as T_r += c_ap Delta with                   */
/* c_ap = 2 pi w_a w_p delta_a sin(theta_p) (both hemispheres folded), so that the */
/* region-averaged angular integral gives                                          */
/*   phi_r = 4 pi qhat_r + T_r / (Sigma_t,r V_r).                                  */
/* Pinned by: pure-absorber attenuation, per-sweep neutron balance, infinite-medium */
/* fixed point, exact-integral agreement on a tiny input.                          */
/* ------------------------------------------------------------------------------ */
static int64_t coarse_slot(const orc_t *o, int i, int j) {
    for (int64_t s = o->nbr_off[i]; s < o->nbr_off[i + 1]; s++)
        if (o->nbr[s] == j) return s;
    return -1;   /* cannot happen: the adjacency was built from these same segments */
}

/* The tracks [t0, t1) of one group sweep, tallied into T_g (and, with a coarse mesh, */
/* the partial currents into jpart [slots][G] and jin [cells][G]).                  */
static void sweep_tracks(orc_t *o, int g, const double *qhat_g, double *T_g, double *jpart, double *jin,
                         int t0, int t1) {
    int P = o->P, G = o->G;
    const int *cell = o->region_cell;
    for (int t = t0; t < t1; t++) {
        int a = o->t_angle[t];
        for (int sense = 0; sense < 2; sense++) {
            for (int p = 0; p < P; p++) {
                double c = 2.0 * ORC_PI * o->wa[a] * o->wp[p] * o->dlt[a] * o->sinp[p];
                size_t idx = (((size_t)t * 2 + sense) * P + p) * G + g;
                double psi = o->psi[idx];
                int64_t n = o->t_off[t + 1] - o->t_off[t];
                int cprev = -1;
                for (int64_t i = 0; i < n; i++) {
                    int64_t k = sense ? o->t_off[t + 1] - 1 - i : o->t_off[t] + i;
                    int r = o->s_reg[k];
                    if (o->n_cells) {
                        /* a coarse-cell boundary crossed with the current psi: the same   */
                        /* weight c turns angular flux into current as Delta into tally    */
                        int ci = cell[r];
                        if (i == 0) jin[(size_t)ci * G + g] += c * psi;
                        else if (ci != cprev) jpart[coarse_slot(o, cprev, ci) * G + g] += c * psi;
                        cprev = ci;
                    }
                    double st = o->sigt[o->region_material[r] * G + g];
                    double tau = st * o->s_len[k] / o->sinp[p];
                    double delta = (psi - qhat_g[r]) * (-expm1(-tau));
                    psi -= delta;
                    T_g[r] += c * delta;
                }
                if (o->n_cells && n > 0) jpart[coarse_slot(o, cprev, -1) * G + g] += c * psi;
                o->psi_exit[idx] = psi;
                int dst = o->link[2 * t + sense];
                if (dst >= 0) {
                    size_t j = ((size_t)dst * P + p) * G + g;
                    if (o->gs_boundary) o->psi[j] = psi;
                    else o->psi_next[j] = psi;
                }
            }
        }
    }
}

/* Threads (a timing convenience; the arithmetic of every track is unchanged). With   */
/* Jacobi boundary updates the tracks of a sweep are independent: thread i takes the  */
/* contiguous track range [i T/n, (i+1) T/n), tallies into private arrays, and the    */
/* arrays are added in thread order afterwards, so a run is reproducible for a given  */
/* thread count, and with one thread every sum is formed in the serial order.         */
/* Boundary Gauss-Seidel runs on one thread.                                          */
int orc_set_threads(orc_t *o, int n) {
    o->nthreads = n > 0 ? n : 1;
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}

static void sweep_group(orc_t *o, int g, const double *qhat_g /* [R] */, double *T_g /* [R] */) {
    int nth = o->nthreads;
    if (nth <= 1 || o->gs_boundary || o->T < 2 * nth) {
        sweep_tracks(o, g, qhat_g, T_g, o->jpart, o->jin_bnd, 0, o->T);
        return;
    }
    int R = o->R, G = o->G;
    size_t nj = o->n_cells ? (size_t)o->nbr_off[o->n_cells] * G : 0;
    size_t ni = o->n_cells ? (size_t)o->n_cells * G : 0;
    size_t per = (size_t)R + nj + ni;
    double *priv = xmalloc(sizeof(double) * per * nth);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nth) schedule(static, 1)
#endif
    for (int i = 0; i < nth; i++) {
        int t0 = (int)((int64_t)o->T * i / nth), t1 = (int)((int64_t)o->T * (i + 1) / nth);
        double *b = priv + per * i;
        sweep_tracks(o, g, qhat_g, b, b + R, b + R + nj, t0, t1);
    }
#ifdef _OPENMP
#pragma omp parallel for num_threads(nth) schedule(static)
#endif
    for (int r = 0; r < R; r++) {
        double v = T_g[r];
        for (int i = 0; i < nth; i++) v += priv[per * i + r];
        T_g[r] = v;
    }
    for (size_t e = 0; e < nj; e++) {
        double v = o->jpart[e];
        for (int i = 0; i < nth; i++) v += priv[per * i + R + e];
        o->jpart[e] = v;
    }
    for (size_t e = 0; e < ni; e++) {
        double v = o->jin_bnd[e];
        for (int i = 0; i < nth; i++) v += priv[per * i + R + nj + e];
        o->jin_bnd[e] = v;
    }
    free(priv);
}

static double sigt_of(const orc_t *o, int r, int g) { return o->sigt[o->region_material[r] * o->G + g]; }

/* Emission density s_{r,g} (Eq. MGNTE, isotropic scattering, per unit volume):    */
/*   s = sum_g' Sigma_s,g'->g phi_g' + chi_g F_r / k (+ external source)           */
/* with F_r = sum_g nuSigma_f,g phi_g.                                             */
static void emission(const orc_t *o, const double *phi, double k, int r, int g, double *s) {
    int G = o->G, m = o->region_material[r];
    double F = 0.0, sc = 0.0;
    for (int gp = 0; gp < G; gp++) {
        F += o->nsf[m * G + gp] * phi[(size_t)r * G + gp];
        sc += o->sigs[((size_t)m * G + gp) * G + g] * phi[(size_t)r * G + gp];
    }
    double v = sc + o->chi[m * G + g] * F / k;
    if (o->qext) v += o->qext[(size_t)r * G + g];
    *s = v;
}

static void swap_psi(orc_t *o) {
    if (o->gs_boundary) return;
    size_t n = (size_t)o->T * 2 * o->P * o->G;
    /* incoming fluxes of unlinked (vacuum) track-senses stay zero */
    double *tmp = o->psi; o->psi = o->psi_next; o->psi_next = tmp;
    memset(o->psi_next, 0, sizeof(double) * n);
}

/* One sweep for a given emission density src [R][G] (per unit volume, all
 * directions): qhat = src / (4 pi Sigma_t); returns phi [R][G] and the tallies.
 * Boundary fluxes are read from, and written back to, the oracle's state. */
void orc_sweep(orc_t *o, const double *src, double *phi_out, double *tally_out) {
    int R = o->R, G = o->G;
    double *q = xmalloc(sizeof(double) * R), *T = xmalloc(sizeof(double) * R);
    if (o->n_cells) {
        memset(o->jpart, 0, sizeof(double) * o->nbr_off[o->n_cells] * G);
        memset(o->jin_bnd, 0, sizeof(double) * (size_t)o->n_cells * G);
    }
    for (int g = 0; g < G; g++) {
        for (int r = 0; r < R; r++) { q[r] = src[(size_t)r * G + g] / (4.0 * ORC_PI * sigt_of(o, r, g)); T[r] = 0.0; }
        sweep_group(o, g, q, T);
        for (int r = 0; r < R; r++) {
            phi_out[(size_t)r * G + g] = 4.0 * ORC_PI * q[r] + T[r] / (sigt_of(o, r, g) * o->V[r]);
            if (tally_out) tally_out[(size_t)r * G + g] = T[r];
        }
    }
    swap_psi(o);
    free(q); free(T);
}

/* ------------------------------------------------------------------------------ */
/* Power (or fixed-source) iteration. Reading (the paper says only "until          */
/* convergence"): start from phi (given, else 1), k (given, else 1), boundary psi  */
/* as stored; every iteration sweeps all groups with the previous iterate's        */
/* source (Jacobi in energy unless gs_energy), updates k <- k * sum V F_new /      */
/* sum V F_old, rescales phi and the boundary psi so that sum V F = 1, and stops   */
/* when ||sqrt(V)(phi_n - phi_n-1)|| / ||sqrt(V) phi_n|| < tol and |dk| < tol.     */
/* With an external source and no normalisation the same loop is a source         */
/* iteration (k fixed to 1).                                                       */
/* ------------------------------------------------------------------------------ */
int orc_solve(orc_t *o, double tol, int max_iter, double *phi /* [R][G] in/out */, double *k_io,
              int *iters, double *resid_out, double *dk_out, int eigen) {
    int R = o->R, G = o->G, P = o->P;
    size_t n = (size_t)R * G;
    double *phin = xmalloc(sizeof(double) * n);
    double *q = xmalloc(sizeof(double) * R), *T = xmalloc(sizeof(double) * R);
    double k = *k_io;
    size_t npsi = (size_t)o->T * 2 * P * G;
    if (eigen) {
        double fs = 0.0;
        for (int r = 0; r < R; r++) {
            int m = o->region_material[r];
            for (int g = 0; g < G; g++) fs += o->V[r] * o->nsf[m * G + g] * phi[(size_t)r * G + g];
        }
        for (size_t i = 0; i < n; i++) phi[i] /= fs;
        for (size_t i = 0; i < npsi; i++) o->psi[i] /= fs;
    }
    int it, conv = 0;
    double res = 1.0, dk = 1.0;
    for (it = 1; it <= max_iter; it++) {
        memcpy(phin, phi, sizeof(double) * n);
        for (int g = 0; g < G; g++) {
            /* Jacobi: source from the previous iterate; energy GS: from the newest */
            const double *src_phi = o->gs_energy ? phin : phi;
            for (int r = 0; r < R; r++) {
                double s;
                emission(o, src_phi, k, r, g, &s);
                if (o->gs_energy) {
                    /* the fission part stays at the previous iterate */
                    int m = o->region_material[r];
                    double F0 = 0.0, F1 = 0.0;
                    for (int gp = 0; gp < G; gp++) {
                        F0 += o->nsf[m * G + gp] * phi[(size_t)r * G + gp];
                        F1 += o->nsf[m * G + gp] * phin[(size_t)r * G + gp];
                    }
                    s += o->chi[m * G + g] * (F0 - F1) / k;
                }
                q[r] = s / (4.0 * ORC_PI * sigt_of(o, r, g));
                T[r] = 0.0;
            }
            sweep_group(o, g, q, T);
            for (int r = 0; r < R; r++)
                phin[(size_t)r * G + g] = 4.0 * ORC_PI * q[r] + T[r] / (sigt_of(o, r, g) * o->V[r]);
        }
        swap_psi(o);
        double knew = k;
        if (eigen) {
            double fs = 0.0;
            for (int r = 0; r < R; r++) {
                int m = o->region_material[r];
                for (int g = 0; g < G; g++) fs += o->V[r] * o->nsf[m * G + g] * phin[(size_t)r * G + g];
            }
            knew = k * fs;
            for (size_t i = 0; i < n; i++) phin[i] /= fs;
            for (size_t i = 0; i < npsi; i++) o->psi[i] /= fs;
        }
        double num = 0.0, den = 0.0;
        for (int r = 0; r < R; r++)
            for (int g = 0; g < G; g++) {
                double d = phin[(size_t)r * G + g] - phi[(size_t)r * G + g];
                num += o->V[r] * d * d;
                den += o->V[r] * phin[(size_t)r * G + g] * phin[(size_t)r * G + g];
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
    free(phin); free(q); free(T);
    return conv ? 0 : 1;
}

/* ------------------------------------------------------------------------------ */
/* Coarse mesh for CMFD (Sec. 2.1.2, Alg. MOCHFEM_CMFD: MOC supplies the currents on  */
/* the radial coarse-cell surfaces). Each region belongs to one coarse cell. The    */
/* surfaces are the ordered cell pairs that some track actually crosses between two */
/* consecutive segments, plus (cell, boundary) where a track enters or leaves the   */
/* domain; every crossing is tallied during the sweep with the flux tally's weight. */
/* Pinned by: per-cell balance of tallies against currents, zero net current across */
/* symmetry planes, and the CMFD fixed point equalling the plain power iteration's. */
/* ------------------------------------------------------------------------------ */
typedef struct { int i, j; } pair_t;
static int cmp_pair(const void *a, const void *b) {
    const pair_t *x = a, *y = b;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return (x->j > y->j) - (x->j < y->j);
}

int orc_set_coarse(orc_t *o, int n_cells, const int *region_cell) {
    free(o->region_cell); free(o->nbr_off); free(o->nbr); free(o->jpart); free(o->jin_bnd);
    o->region_cell = NULL; o->nbr_off = NULL; o->nbr = NULL; o->jpart = NULL; o->jin_bnd = NULL;
    o->n_cells = 0;
    if (n_cells <= 0) return 0;
    for (int r = 0; r < o->R; r++)
        if (region_cell[r] < 0 || region_cell[r] >= n_cells) return 1;
    o->region_cell = xmalloc(sizeof(int) * o->R);
    memcpy(o->region_cell, region_cell, sizeof(int) * o->R);
    size_t cap = 1024, np = 0;
    pair_t *pr = xmalloc(sizeof(pair_t) * cap);
    for (int t = 0; t < o->T; t++) {
        int64_t k0 = o->t_off[t], k1 = o->t_off[t + 1];
        if (k1 == k0) continue;
        for (int64_t k = k0; k <= k1; k++) {
            int ci = k == k0 ? -1 : region_cell[o->s_reg[k - 1]];
            int cj = k == k1 ? -1 : region_cell[o->s_reg[k]];
            if (ci == cj) continue;
            if (np + 2 > cap) { cap *= 2; pr = realloc(pr, sizeof(pair_t) * cap); }
            /* both orientations: each surface is listed under both of its cells */
            if (ci >= 0) pr[np++] = (pair_t){ci, cj};
            if (cj >= 0) pr[np++] = (pair_t){cj, ci};
        }
    }
    qsort(pr, np, sizeof(pair_t), cmp_pair);
    size_t nu = 0;
    for (size_t i = 0; i < np; i++)
        if (nu == 0 || cmp_pair(&pr[i], &pr[nu - 1]) != 0) pr[nu++] = pr[i];
    o->n_cells = n_cells;
    o->nbr_off = xmalloc(sizeof(int64_t) * (n_cells + 1));
    o->nbr = xmalloc(sizeof(int) * (nu ? nu : 1));
    for (size_t i = 0; i < nu; i++) { o->nbr[i] = pr[i].j; o->nbr_off[pr[i].i + 1]++; }
    for (int c = 0; c < n_cells; c++) o->nbr_off[c + 1] += o->nbr_off[c];
    free(pr);
    o->jpart = xmalloc(sizeof(double) * (nu ? nu : 1) * o->G);
    o->jin_bnd = xmalloc(sizeof(double) * (size_t)n_cells * o->G);
    return 0;
}
int64_t orc_coarse_slots(const orc_t *o) { return o->n_cells ? o->nbr_off[o->n_cells] : 0; }
void orc_coarse_adjacency(const orc_t *o, int64_t *off, int *nbr) {
    memcpy(off, o->nbr_off, sizeof(int64_t) * (o->n_cells + 1));
    memcpy(nbr, o->nbr, sizeof(int) * o->nbr_off[o->n_cells]);
}
void orc_currents(const orc_t *o, double *jpart, double *jin_bnd) {
    memcpy(jpart, o->jpart, sizeof(double) * o->nbr_off[o->n_cells] * o->G);
    memcpy(jin_bnd, o->jin_bnd, sizeof(double) * (size_t)o->n_cells * o->G);
}
