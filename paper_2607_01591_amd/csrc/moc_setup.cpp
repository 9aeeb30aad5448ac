// Host setup of libmoc: half-edge mesh, cyclic track laydown, ray tracing by mesh walk,
// boundary links. Follows the paper's Sec. 3.1: a half-edge data structure for the 2D
// mesh, modular rays laid on the bounding box of the whole domain, and ray-mesh
// intersection by traversing the half-edge structure to obtain (length, element) per
// segment.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <functional>
#include <climits>
#include <thread>
#include <unordered_map>

#include "moc_internal.h"

namespace moc {

static constexpr double kPi = 3.14159265358979323846;

void parallel_for(int64_t n, int nthreads, int64_t chunk, const std::function<void(int64_t, int64_t, int)> &f) {
    if (nthreads <= 1 || n <= chunk) {
        f(0, n, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> errs(nthreads);
    for (int w = 0; w < nthreads; ++w) {
        th.emplace_back([&, w] {
            try {
                for (;;) {
                    int64_t b = next.fetch_add(chunk);
                    if (b >= n) break;
                    f(b, std::min(n, b + chunk), w);
                }
            } catch (...) {
                errs[w] = std::current_exception();
            }
        });
    }
    for (auto &t : th) t.join();
    for (auto &e : errs)
        if (e) std::rethrow_exception(e);
}

// ---------------------------------------------------------------- mesh
// Side s of the domain as a line: points p with n_s . p = c_s (outward normal n_s),
// and a direction along it for ordering.
static void side_line(const Mesh &m, int s, double &nx, double &ny, double &c, double &tx, double &ty) {
    if (m.domain == MOC_DOMAIN_BOX) {
        static const double N[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
        nx = N[s][0];
        ny = N[s][1];
        const double v[4] = {-m.box[0], m.box[2], -m.box[1], m.box[3]};
        c = v[s];
    } else {
        const double ang = (30.0 + 60.0 * s) * kPi / 180.0;
        const double cx = 0.5 * (m.box[0] + m.box[2]), cy = 0.5 * (m.box[1] + m.box[3]);
        nx = std::cos(ang);
        ny = std::sin(ang);
        c = nx * cx + ny * cy + m.hex_apothem;
    }
    tx = -ny;
    ty = nx;
}

void build_mesh(const moc_mesh &in, Mesh &m) {
    if (in.n_vertices <= 0 || in.n_triangles <= 0 || in.n_regions <= 0 || !in.xy || !in.tri ||
        !in.tri_region)
        throw Error(MOC_EINVAL, "mesh: empty or null arrays");
    if (in.domain != MOC_DOMAIN_BOX && in.domain != MOC_DOMAIN_HEXAGON)
        throw Error(MOC_EINVAL, "mesh: unknown domain kind");
    m.nv = in.n_vertices;
    m.nt = in.n_triangles;
    m.R = in.n_regions;
    m.xy.assign(in.xy, in.xy + 2 * (size_t)m.nv);
    m.tri.assign(in.tri, in.tri + 3 * (size_t)m.nt);
    m.tri_region.assign(in.tri_region, in.tri_region + m.nt);
    m.domain = in.domain;
    for (int i = 0; i < 4; ++i) m.box[i] = in.box[i];
    m.hex_apothem = in.hex_apothem;
    m.n_sides = m.domain == MOC_DOMAIN_BOX ? 4 : 6;
    for (int i = 0; i < m.n_sides; ++i) {
        if (in.bc[i] != MOC_BC_VACUUM && in.bc[i] != MOC_BC_REFLECTIVE)
            throw Error(MOC_EINVAL, "mesh: unknown boundary condition");
        m.bc[i] = in.bc[i];
        if (m.domain == MOC_DOMAIN_HEXAGON && in.bc[i] != MOC_BC_VACUUM)
            throw Error(MOC_EINVAL, "mesh: hexagonal domains support vacuum boundaries only");
    }
    if (!(m.box[2] > m.box[0] && m.box[3] > m.box[1])) throw Error(MOC_EINVAL, "mesh: empty bounding box");
    std::vector<char> used(m.R, 0);
    for (int t = 0; t < m.nt; ++t) {
        const int *v = &m.tri[3 * (size_t)t];
        for (int k = 0; k < 3; ++k)
            if (v[k] < 0 || v[k] >= m.nv) throw Error(MOC_EINVAL, "mesh: vertex index out of range");
        const double *a = &m.xy[2 * (size_t)v[0]], *b = &m.xy[2 * (size_t)v[1]], *c = &m.xy[2 * (size_t)v[2]];
        const double area2 = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
        if (!(area2 > 0)) throw Error(MOC_EINVAL, "mesh: triangle " + std::to_string(t) + " is not counter-clockwise");
        const int r = m.tri_region[t];
        if (r < 0 || r >= m.R) throw Error(MOC_EINVAL, "mesh: region index out of range");
        used[r] = 1;
    }
    for (int r = 0; r < m.R; ++r)
        if (!used[r]) throw Error(MOC_EINVAL, "mesh: region " + std::to_string(r) + " has no triangle");
    // twins: sort directed edges by (from, to); the twin of u->v is v->u
    const size_t ne = 3 * (size_t)m.nt;
    std::vector<std::pair<uint64_t, int>> keys(ne);
    for (size_t h = 0; h < ne; ++h) {
        const int t = int(h / 3), e = int(h % 3);
        const uint64_t u = (uint32_t)m.tri[3 * (size_t)t + e], v = (uint32_t)m.tri[3 * (size_t)t + (e + 1) % 3];
        keys[h] = {(u << 32) | v, int(h)};
    }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 1; i < ne; ++i)
        if (keys[i].first == keys[i - 1].first) throw Error(MOC_EINVAL, "mesh: non-manifold or inconsistently oriented edge");
    m.twin.assign(ne, -1);
    for (size_t h = 0; h < ne; ++h) {
        const uint64_t k = keys[h].first;
        const uint64_t rev = (k << 32) | (k >> 32);
        auto it = std::lower_bound(keys.begin(), keys.end(), std::make_pair(rev, -1));
        if (it != keys.end() && it->first == rev) m.twin[keys[h].second] = it->second;
    }
    // boundary half-edges must lie on a domain side
    m.side_edges.assign(m.n_sides, {});
    const double scale = (m.box[2] - m.box[0]) + (m.box[3] - m.box[1]);
    const double tol = 1e-9 * scale;
    for (size_t h = 0; h < ne; ++h) {
        if (m.twin[h] >= 0) continue;
        const int t = int(h / 3), e = int(h % 3);
        const double *p = &m.xy[2 * (size_t)m.tri[3 * (size_t)t + e]];
        const double *q = &m.xy[2 * (size_t)m.tri[3 * (size_t)t + (e + 1) % 3]];
        int side = -1;
        for (int s = 0; s < m.n_sides && side < 0; ++s) {
            double nx, ny, c, tx, ty;
            side_line(m, s, nx, ny, c, tx, ty);
            if (std::fabs(nx * p[0] + ny * p[1] - c) < tol && std::fabs(nx * q[0] + ny * q[1] - c) < tol) {
                side = s;
                const double a = tx * p[0] + ty * p[1], b = tx * q[0] + ty * q[1];
                m.side_edges[s].push_back({std::min(a, b), int(h)});
            }
        }
        if (side < 0) throw Error(MOC_EINVAL, "mesh: a boundary edge does not lie on the domain boundary");
    }
    for (auto &v : m.side_edges) std::sort(v.begin(), v.end());
}

// ---------------------------------------------------------------- quadrature
// Half-range Gauss-Legendre by Newton iteration on the Legendre recurrence (the positive
// roots of P_{2n}); weights of one hemisphere sum to one.
static void gauss_legendre_half(int n, std::vector<double> &mu, std::vector<double> &w) {
    const int N = 2 * n;
    mu.resize(n);
    w.resize(n);
    auto legendre = [N](double x, double &pn, double &dpn) {
        double a = 1.0, b = x;
        for (int k = 2; k <= N; ++k) {
            const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
            a = b;
            b = c;
        }
        pn = b;
        dpn = N * (x * b - a) / (x * x - 1.0);
    };
    for (int i = 0; i < n; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double pn, dpn;
            legendre(x, pn, dpn);
            const double dx = pn / dpn;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double pn, dpn;
        legendre(x, pn, dpn);
        mu[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dpn * dpn);
    }
}

void build_quadrature(const Mesh &m, const moc_tracks &tr, Quadrature &q) {
    if (tr.n_azim <= 0 || tr.n_azim % 4) throw Error(MOC_EINVAL, "tracks: n_azim must be a positive multiple of 4");
    if (tr.n_polar < 1 || tr.n_polar > kMaxPolar) throw Error(MOC_EINVAL, "tracks: n_polar must be in 1..4");
    if (!(tr.spacing > 0)) throw Error(MOC_EINVAL, "tracks: spacing must be positive");
    q.A = tr.n_azim;
    q.NA = tr.n_azim / 2;
    q.P = tr.n_polar;
    const double W = m.box[2] - m.box[0], H = m.box[3] - m.box[1];
    const int NQ = q.A / 4;
    q.phi.assign(q.NA, 0);
    q.delta.assign(q.NA, 0);
    q.wa.assign(q.NA, 0);
    q.nx.assign(q.NA, 0);
    q.ny.assign(q.NA, 0);
    // cyclic correction on the bounding box: an integer number of track crossings on
    // each side so that track ends coincide under reflection
    for (int a = 0; a < NQ; ++a) {
        const double nominal = 2.0 * kPi * (a + 0.5) / q.A;
        const int nx = (int)std::ceil(W * std::sin(nominal) / tr.spacing);
        const int ny = (int)std::ceil(H * std::cos(nominal) / tr.spacing);
        const double phi = std::atan((H * nx) / (W * ny));
        const double d = (W / nx) * std::sin(phi);
        const int b = q.NA - 1 - a;
        q.phi[a] = phi;
        q.phi[b] = kPi - phi;
        q.delta[a] = q.delta[b] = d;
        q.nx[a] = q.nx[b] = nx;
        q.ny[a] = q.ny[b] = ny;
    }
    for (int a = 0; a < q.NA; ++a) {
        const double lo = a == 0 ? 0.0 : 0.5 * (q.phi[a - 1] + q.phi[a]);
        const double hi = a == q.NA - 1 ? kPi : 0.5 * (q.phi[a] + q.phi[a + 1]);
        q.wa[a] = (hi - lo) / kPi;
    }
    if (tr.polar_mu) {
        if (!tr.polar_w) throw Error(MOC_EINVAL, "tracks: polar_w required with polar_mu");
        q.mu.assign(tr.polar_mu, tr.polar_mu + q.P);
        q.wp.assign(tr.polar_w, tr.polar_w + q.P);
        for (int p = 0; p < q.P; ++p)
            if (!(q.mu[p] >= 0 && q.mu[p] < 1 && q.wp[p] > 0)) throw Error(MOC_EINVAL, "tracks: bad polar quadrature");
    } else {
        gauss_legendre_half(q.P, q.mu, q.wp);
    }
    q.sinp.resize(q.P);
    for (int p = 0; p < q.P; ++p) q.sinp[p] = std::sqrt(1.0 - q.mu[p] * q.mu[p]);
}

// ---------------------------------------------------------------- tracks
// Clip the line p + s u to the domain; returns false if it misses. side_in receives the
// side through which it enters.
static bool clip_domain(const Mesh &m, double px, double py, double ux, double uy, double &s0, double &s1,
                        int &side_in) {
    s0 = -1e300;
    s1 = 1e300;
    side_in = -1;
    for (int s = 0; s < m.n_sides; ++s) {
        double nx, ny, c, tx, ty;
        side_line(m, s, nx, ny, c, tx, ty);
        const double den = nx * ux + ny * uy;       // > 0: leaving through this side
        const double num = c - (nx * px + ny * py);  // >= 0 inside
        if (den == 0.0) {
            if (num < 0) return false;
            continue;
        }
        const double s_hit = num / den;
        if (den > 0) {
            s1 = std::min(s1, s_hit);
        } else if (s_hit > s0) {
            s0 = s_hit;
            side_in = s;
        }
    }
    return s1 - s0 > 1e-12;
}

void lay_tracks(const Mesh &m, const Quadrature &q, Tracks &t) {
    const double W = m.box[2] - m.box[0], H = m.box[3] - m.box[1];
    t = Tracks();
    for (int a = 0; a < q.NA; ++a) {
        const double ux = std::cos(q.phi[a]), uy = std::sin(q.phi[a]);
        // starting points: bottom side, then the left (phi < pi/2) or right side; all
        // tracks of one angle are parallel lines spaced by delta_a
        std::vector<std::pair<double, std::pair<double, double>>> st;
        for (int i = 0; i < q.nx[a]; ++i) {
            const double x = m.box[0] + (i + 0.5) * W / q.nx[a], y = m.box[1];
            st.push_back({-uy * x + ux * y, {x, y}});
        }
        for (int j = 0; j < q.ny[a]; ++j) {
            const double x = ux > 0 ? m.box[0] : m.box[2], y = m.box[1] + (j + 0.5) * H / q.ny[a];
            st.push_back({-uy * x + ux * y, {x, y}});
        }
        std::sort(st.begin(), st.end(), [](const auto &l, const auto &r) { return l.first < r.first; });
        for (auto &e : st) {
            const double px = e.second.first, py = e.second.second;
            double s0, s1;
            int side;
            if (!clip_domain(m, px, py, ux, uy, s0, s1, side)) continue;
            t.angle.push_back(a);
            t.x0.push_back(px + s0 * ux);
            t.y0.push_back(py + s0 * uy);
            t.x1.push_back(px + s1 * ux);
            t.y1.push_back(py + s1 * uy);
            t.len.push_back(s1 - s0);
            t.entry_side.push_back(side);
        }
    }
    t.T = (int)t.angle.size();
}

// Reflective links by matching quantised boundary positions in a hash map: the exit of
// a track-sense on a reflective side feeds the track-sense that starts at the same
// point in the mirrored direction. Vacuum exits get -1.
void link_tracks(const Mesh &m, const Quadrature &q, Tracks &t) {
    t.link.assign(2 * (size_t)t.T, -1);
    bool any_reflective = false;
    for (int s = 0; s < m.n_sides; ++s) any_reflective |= m.bc[s] == MOC_BC_REFLECTIVE;
    if (!any_reflective) return;
    double dmin = 1e300;
    for (double d : q.delta) dmin = std::min(dmin, d);
    const double quantum = dmin * 1e-3;
    auto side_of = [&](double x, double y) {
        const double tol = 1e-9 * ((m.box[2] - m.box[0]) + (m.box[3] - m.box[1]));
        if (std::fabs(x - m.box[0]) < tol) return 0;
        if (std::fabs(x - m.box[2]) < tol) return 1;
        if (std::fabs(y - m.box[1]) < tol) return 2;
        if (std::fabs(y - m.box[3]) < tol) return 3;
        return -1;
    };
    // key: side, quantised position along the side, track angle of the start and its
    // direction quadrant (tracks of different angles can share a boundary point; the
    // mirror image of track angle a is track angle NA - 1 - a)
    auto key = [&](int side, double pos, int angle, double dx, double dy) -> int64_t {
        const int64_t qp = (int64_t)std::llround(pos / quantum);
        const int quad = (dx > 0 ? 1 : 0) | (dy > 0 ? 2 : 0);
        return ((qp * 4 + side) * q.NA + angle) * 4 + quad;
    };
    std::unordered_map<int64_t, int> starts;
    starts.reserve(4 * (size_t)t.T);
    for (int i = 0; i < t.T; ++i) {
        const double ux = std::cos(q.phi[t.angle[i]]), uy = std::sin(q.phi[t.angle[i]]);
        for (int s = 0; s < 2; ++s) {
            const double x = s ? t.x1[i] : t.x0[i], y = s ? t.y1[i] : t.y0[i];
            const int sd = side_of(x, y);
            if (sd < 0) throw Error(MOC_EINVAL, "tracks: track end is not on the box");
            const double pos = sd < 2 ? y : x;
            starts[key(sd, pos, t.angle[i], s ? -ux : ux, s ? -uy : uy)] = 2 * i + s;
        }
    }
    for (int i = 0; i < t.T; ++i) {
        const double ux = std::cos(q.phi[t.angle[i]]), uy = std::sin(q.phi[t.angle[i]]);
        for (int s = 0; s < 2; ++s) {
            const double x = s ? t.x0[i] : t.x1[i], y = s ? t.y0[i] : t.y1[i];
            const int sd = side_of(x, y);
            if (m.bc[sd] != MOC_BC_REFLECTIVE) continue;
            double dx = s ? -ux : ux, dy = s ? -uy : uy;
            if (sd < 2) dx = -dx; else dy = -dy;
            const double pos = sd < 2 ? y : x;
            const int mirror = q.NA - 1 - t.angle[i];
            auto it = starts.find(key(sd, pos, mirror, dx, dy));
            if (it == starts.end()) {
                // tolerate a position that rounds to the neighbouring quantum
                const double fr = pos / quantum - std::floor(pos / quantum);
                const double d2 = pos + (fr < 0.5 ? 0.5 : -0.5) * quantum;
                it = starts.find(key(sd, d2, mirror, dx, dy));
            }
            if (it == starts.end()) throw Error(MOC_EINVAL, "tracks: no reflected partner found (cyclic laydown broken)");
            t.link[2 * (size_t)i + s] = it->second;
        }
    }
}

// ---------------------------------------------------------------- ray tracing
// Find the boundary half-edge of `side` containing the point at parameter `pos`.
static int locate_boundary_edge(const Mesh &m, int side, double px, double py) {
    double nx, ny, c, tx, ty;
    side_line(m, side, nx, ny, c, tx, ty);
    const double pos = tx * px + ty * py;
    const auto &v = m.side_edges[side];
    // the same tolerance that admitted the edges to this side: a mesh corner vertex may sit
    // that far from the exact corner, where tracks through the corner enter
    const double tol = 1e-9 * ((m.box[2] - m.box[0]) + (m.box[3] - m.box[1]));
    const size_t ub = size_t(std::upper_bound(v.begin(), v.end(), std::make_pair(pos, INT32_MAX)) - v.begin());
    // candidates: the edge starting at or before pos, the one before it, and the first edge
    const size_t cand[3] = {ub >= 1 ? ub - 1 : v.size(), ub >= 2 ? ub - 2 : v.size(), 0};
    for (size_t ci : cand) {
        if (ci >= v.size()) continue;
        const int h = v[ci].second;
        const int t = h / 3, e = h % 3;
        const double *p = &m.xy[2 * (size_t)m.tri[3 * (size_t)t + e]];
        const double *q = &m.xy[2 * (size_t)m.tri[3 * (size_t)t + (e + 1) % 3]];
        const double a = tx * p[0] + ty * p[1], b = tx * q[0] + ty * q[1];
        const double lo = std::min(a, b), hi = std::max(a, b);
        if (pos >= lo - tol && pos <= hi + tol) return h;
    }
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "tracking: entry point (%.17g, %.17g) not on any boundary edge of side %d "
                  "(mesh does not cover the domain; %zu edges on that side)", px, py, side, v.size());
    throw Error(MOC_EINVAL, msg);
}

int64_t trace_track(const Mesh &m, const Quadrature &q, const Tracks &tk, int track, SegmentSink &sink) {
    const double ux = std::cos(q.phi[tk.angle[track]]), uy = std::sin(q.phi[tk.angle[track]]);
    const double ox = tk.x0[track], oy = tk.y0[track], L = tk.len[track];
    int he = locate_boundary_edge(m, tk.entry_side[track], ox, oy);
    int tri = he / 3;
    double s = 0.0;
    int cur_reg = -1;
    double cur_len = 0.0;
    int64_t nseg = 0;
    const int max_steps = 4 * m.nt + 16;
    for (int step = 0; step < max_steps; ++step) {
        // exit edge: the smallest crossing parameter over edges the ray leaves through,
        // other than the entry edge
        const int *v = &m.tri[3 * (size_t)tri];
        double best = 1e300;
        int best_e = -1;
        for (int e = 0; e < 3; ++e) {
            if (3 * tri + e == he) continue;
            const double *p = &m.xy[2 * (size_t)v[e]];
            const double *qq = &m.xy[2 * (size_t)v[(e + 1) % 3]];
            const double nx = qq[1] - p[1], ny = -(qq[0] - p[0]);  // outward for CCW
            const double den = nx * ux + ny * uy;
            if (den <= 0) continue;
            const double se = (nx * (p[0] - ox) + ny * (p[1] - oy)) / den;
            if (se < best) {
                best = se;
                best_e = e;
            }
        }
        if (best_e < 0) throw Error(MOC_EINVAL, "tracking: ray cannot leave a triangle (degenerate mesh)");
        const double s_exit = std::max(best, s);
        const double piece = s_exit - s;
        if (piece >= 1e-12) {   // drop tiny pieces first, then merge same-region runs
            const int r = m.tri_region[tri];
            if (r == cur_reg) {
                cur_len += piece;
            } else {
                if (cur_reg >= 0) {
                    sink.emit(cur_reg, cur_len);
                    ++nseg;
                }
                cur_reg = r;
                cur_len = piece;
            }
        }
        s = s_exit;
        const int out = 3 * tri + best_e;
        const int nxt = m.twin[out];
        if (nxt < 0) {
            if (std::fabs(s - L) > 1e-9 * (1.0 + L))
                throw Error(MOC_EINVAL, "tracking: ray left the mesh before the domain boundary");
            break;
        }
        he = nxt;
        tri = nxt / 3;
        if (step == max_steps - 1) throw Error(MOC_EINVAL, "tracking: walk did not terminate");
    }
    if (cur_reg >= 0) {
        sink.emit(cur_reg, cur_len);
        ++nseg;
    }
    return nseg;
}

// ---------------------------------------------------------------- locality
static inline uint64_t spread16(uint64_t x) {
    x &= 0xffff;
    x = (x | (x << 8)) & 0x00ff00ffULL;
    x = (x | (x << 4)) & 0x0f0f0f0fULL;
    x = (x | (x << 2)) & 0x33333333ULL;
    x = (x | (x << 1)) & 0x55555555ULL;
    return x;
}

void locality_order(const Mesh &m, std::vector<int> &internal_of_user, std::vector<int> &user_of_internal) {
    std::vector<double> cx(m.R, 0), cy(m.R, 0), w(m.R, 0);
    for (int t = 0; t < m.nt; ++t) {
        const int *v = &m.tri[3 * (size_t)t];
        const double *a = &m.xy[2 * (size_t)v[0]], *b = &m.xy[2 * (size_t)v[1]], *c = &m.xy[2 * (size_t)v[2]];
        const double ar = 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]));
        const int r = m.tri_region[t];
        cx[r] += ar * (a[0] + b[0] + c[0]) / 3;
        cy[r] += ar * (a[1] + b[1] + c[1]) / 3;
        w[r] += ar;
    }
    const double W = m.box[2] - m.box[0], H = m.box[3] - m.box[1];
    std::vector<std::pair<uint64_t, int>> key(m.R);
    for (int r = 0; r < m.R; ++r) {
        const double x = (cx[r] / w[r] - m.box[0]) / W, y = (cy[r] / w[r] - m.box[1]) / H;
        const uint64_t ix = (uint64_t)std::min(65535.0, std::max(0.0, x * 65536.0));
        const uint64_t iy = (uint64_t)std::min(65535.0, std::max(0.0, y * 65536.0));
        key[r] = {spread16(ix) | (spread16(iy) << 1), r};
    }
    std::sort(key.begin(), key.end());
    internal_of_user.resize(m.R);
    user_of_internal.resize(m.R);
    for (int i = 0; i < m.R; ++i) {
        user_of_internal[i] = key[i].second;
        internal_of_user[key[i].second] = i;
    }
}

}  // namespace moc
