// C ABI of libmoc's DFEM-SN solver (declared in include/dfem.h): host setup (mesh,
// element and face matrices in closed form, direction set, dependency levels, the
// compressed angular-flux storage of Alg. DFEM_SN_sweep), the sweep as one launch per
// dependency level, and the power / source iteration. No exception crosses the ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <thread>

#include "dfem.h"
#include "dfem_kernels.h"
#include "moc_internal.h"

using namespace moc;

#define SN_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) throw Error(MOC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// host data the tiled schedule is built from (kept after create)
struct SnHost {
    int T = 0, A = 0, P = 0, nd = 0;
    std::vector<int> nbr;          // [T][3] neighbour element, or -1 - side
    std::vector<double> nrm;       // [T][3][2] outward unit normals (FP64)
    std::vector<double> azc, azs;  // azimuths' unit in-plane vectors
    std::vector<int> bface;        // [3T] boundary face index, or -1
    std::vector<int> rx, ry;       // mirrored directions
    int bc[6] = {0, 0, 0, 0, 0, 0};
    // inflow / outflow by the sign of Omega . n taken with the azimuth's unit vector (as
    // for the level schedule, so both agree on every face)
    double onf(int dd, int e, int k) const {
        const int a = dd / P;
        return azc[a] * nrm[((size_t)e * 3 + k) * 2] + azs[a] * nrm[((size_t)e * 3 + k) * 2 + 1];
    }
};

struct moc_sn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevSN d;
    SnHost h;
    DevSNTiles tl;
    bool tiled = false;            // sweeps use the tiled schedule
    std::vector<void *> tile_allocs;
    int max_iter = 10000, check_every = 1, n_threads = 1;
    bool fissile = false, fixed_source = false;
    bool host_only = false;   // negative device ordinal: host setup and its checks only
    int cur_phi = 0, cur_bnd = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // the sweep's launches, one per boundary-buffer parity
    double setup_ms = 0;
    int64_t device_bytes = 0;
    double *host_scal = nullptr;
    std::vector<std::pair<void *, size_t>> allocs;
    std::string err;
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_pool;
    int64_t prof_n = 0;
    double prof_ms = 0, prof_min = 0, prof_max = 0;

    template <typename T> T *dalloc(size_t n) {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(n * sizeof(T), 16);
        if (hipMalloc(&p, bytes) != hipSuccess) throw Error(MOC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        allocs.push_back({p, bytes});
        device_bytes += (int64_t)bytes;
        return (T *)p;
    }
    template <typename T> T *upload(const std::vector<T> &v) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) SN_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    void dfree(void *p) {
        for (size_t i = 0; i < allocs.size(); ++i)
            if (allocs[i].first == p) {
                (void)hipFree(p);
                device_bytes -= (int64_t)allocs[i].second;
                allocs.erase(allocs.begin() + (long)i);
                return;
            }
    }
    ~moc_sn_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto *v : {&prof_pending, &prof_pool})
            for (auto &e : *v) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        for (auto &a : allocs) (void)hipFree(a.first);
        if (host_scal) (void)hipHostFree(host_scal);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

static thread_local std::string g_sn_create_error;

static int sn_guarded(moc_sn_ctx *c, const std::function<void()> &f) {
    try {
        f();
        if (c) c->err.clear();
        return MOC_OK;
    } catch (const Error &e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return MOC_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        return MOC_EINVAL;
    }
}

static void sn_create_impl(const moc_mesh *mesh_in, const moc_tracks *angles, const moc_xs *xs, const moc_options *opt,
                           moc_sn_ctx *c) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!mesh_in || !angles || !xs) throw Error(MOC_EINVAL, "sn create: null argument");
    moc_options o{};
    if (opt) o = *opt;
    if (o.precision != MOC_PREC_F32 && o.precision != MOC_PREC_F64) throw Error(MOC_EINVAL, "options: bad precision");
    if (mesh_in->domain != MOC_DOMAIN_BOX) throw Error(MOC_EINVAL, "sn create: box domains only");
    c->max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    c->check_every = o.check_every > 0 ? o.check_every : 1;
    c->n_threads = o.n_threads > 0 ? o.n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    const int M = xs->n_materials, G = xs->n_groups;
    if (M <= 0 || G <= 0 || !xs->sigma_t || !xs->sigma_s || !xs->nu_sigma_f || !xs->chi)
        throw Error(MOC_EINVAL, "xs: empty or null arrays");
    for (int i = 0; i < M * G; ++i)
        if (!(xs->sigma_t[i] > 0) || !std::isfinite(xs->sigma_t[i])) throw Error(MOC_EINVAL, "xs: Sigma_t must be positive and finite");
    if (!mesh_in->region_material) throw Error(MOC_EINVAL, "mesh: null region_material");
    Mesh m;
    build_mesh(*mesh_in, m);
    for (int r = 0; r < m.R; ++r)
        if (mesh_in->region_material[r] < 0 || mesh_in->region_material[r] >= M)
            throw Error(MOC_EINVAL, "mesh: material index out of range");
    moc_tracks tr = *angles;
    if (!(tr.spacing > 0)) tr.spacing = 1.0;   // the polar set does not depend on it
    Quadrature quad;
    build_quadrature(m, tr, quad);
    for (int i = 0; i < M * G; ++i) c->fissile |= xs->nu_sigma_f[i] > 0;

    DevSN &d = c->d;
    const int T = m.nt, A = quad.A, P = quad.P, nd = A * P;
    d.T = T;
    d.G = G;
    d.M = M;
    d.nd = nd;
    d.precision = o.precision;
    const bool f64 = o.precision == MOC_PREC_F64;

    // ---- directions: product of equally spaced azimuths and the polar set
    std::vector<double> dirs((size_t)nd * 3);
    std::vector<int> rx(nd), ry(nd);
    for (int a = 0; a < A; ++a) {
        const double ph = 2.0 * 3.14159265358979323846 * (a + 0.5) / A;
        for (int p = 0; p < P; ++p) {
            const int k = a * P + p;
            dirs[3 * k] = quad.sinp[p] * std::cos(ph);
            dirs[3 * k + 1] = quad.sinp[p] * std::sin(ph);
            dirs[3 * k + 2] = 4.0 * 3.14159265358979323846 * quad.wp[p] / A;
            rx[k] = ((A / 2 - 1 - a + A) % A) * P + p;   // mirror across a side normal to x: phi -> pi - phi
            ry[k] = (A - 1 - a) * P + p;                  // across a side normal to y: phi -> -phi
        }
    }

    // ---- element geometry and matrices in closed form (FP64)
    std::vector<double> area(T), mass((size_t)T * 6), mass9((size_t)T * 9), fmass((size_t)T * 18), fcpl((size_t)T * 27, 0.0),
        nrm((size_t)T * 6), gradw(T), cx(T), cy(T), L(T);
    std::vector<int> nbr((size_t)T * 3), side_of_half(3 * (size_t)T, -1);
    for (int s = 0; s < m.n_sides; ++s)
        for (auto &pe : m.side_edges[s]) side_of_half[pe.second] = s;
    for (int e = 0; e < T; ++e) {
        const double *v[3];
        for (int k = 0; k < 3; ++k) v[k] = &m.xy[2 * (size_t)m.tri[3 * (size_t)e + k]];
        area[e] = 0.5 * ((v[1][0] - v[0][0]) * (v[2][1] - v[0][1]) - (v[2][0] - v[0][0]) * (v[1][1] - v[0][1]));
        cx[e] = (v[0][0] + v[1][0] + v[2][0]) / 3.0;
        cy[e] = (v[0][1] + v[1][1] + v[2][1]) / 3.0;
        L[e] = std::sqrt(area[e]);
    }
    auto basis_at = [&](int e, const double *p, double *u) {
        u[0] = 1.0;
        u[1] = (p[0] - cx[e]) / L[e];
        u[2] = (p[1] - cy[e]) / L[e];
    };
    for (int e = 0; e < T; ++e) {
        const double *v[3];
        for (int k = 0; k < 3; ++k) v[k] = &m.xy[2 * (size_t)m.tri[3 * (size_t)e + k]];
        // second moments about the centroid: int (x - x_c)^2 = area / 12 sum_k (x_k - x_c)^2, etc.
        double sxx = 0, sxy = 0, syy = 0;
        for (int k = 0; k < 3; ++k) {
            const double dx = v[k][0] - cx[e], dy = v[k][1] - cy[e];
            sxx += dx * dx;
            sxy += dx * dy;
            syy += dy * dy;
        }
        const double l2 = L[e] * L[e];
        const double M9[9] = {area[e], 0.0, 0.0, 0.0, area[e] * sxx / (12.0 * l2), area[e] * sxy / (12.0 * l2),
                              0.0, area[e] * sxy / (12.0 * l2), area[e] * syy / (12.0 * l2)};
        for (int i = 0; i < 9; ++i) mass9[(size_t)e * 9 + i] = M9[i];
        const double ms[6] = {M9[0], M9[1], M9[2], M9[4], M9[5], M9[8]};
        for (int i = 0; i < 6; ++i) mass[(size_t)e * 6 + i] = ms[i];
        gradw[e] = area[e] / L[e];
        for (int k = 0; k < 3; ++k) {
            const double *pa = v[k], *pb = v[(k + 1) % 3];
            const double tx = pb[0] - pa[0], ty = pb[1] - pa[1], len = std::sqrt(tx * tx + ty * ty);
            nrm[((size_t)e * 3 + k) * 2] = ty / len;
            nrm[((size_t)e * 3 + k) * 2 + 1] = -tx / len;
            const int h = 3 * e + k, tw = m.twin[h];
            nbr[(size_t)e * 3 + k] = tw >= 0 ? tw / 3 : -1 - side_of_half[h];
            // along the edge u(s) = alpha + s beta, s in [0, 1]:
            // int u_j v_i = len (alpha_j alpha'_i + (alpha_j beta'_i + beta_j alpha'_i) / 2 + beta_j beta'_i / 3)
            double ua[3], ub[3];
            basis_at(e, pa, ua);
            basis_at(e, pb, ub);
            auto edge_int = [&](const double *aa, const double *bb, const double *a2, const double *b2, int j, int i) {
                const double al = aa[j], be = bb[j] - aa[j], al2 = a2[i], be2 = b2[i] - a2[i];
                return len * (al * al2 + 0.5 * (al * be2 + be * al2) + be * be2 / 3.0);
            };
            const int sidx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
            for (int q = 0; q < 6; ++q)
                fmass[((size_t)e * 3 + k) * 6 + q] = edge_int(ua, ub, ua, ub, sidx[q][0], sidx[q][1]);
            if (tw >= 0) {
                double na[3], nb[3];
                basis_at(tw / 3, pa, na);
                basis_at(tw / 3, pb, nb);
                for (int j = 0; j < 3; ++j)
                    for (int i = 0; i < 3; ++i) fcpl[((size_t)e * 3 + k) * 9 + 3 * j + i] = edge_int(ua, ub, na, nb, j, i);
            }
        }
    }
    for (int h = 0; h < 3 * T; ++h)
        if (m.twin[h] < 0 && side_of_half[h] < 0) throw Error(MOC_EINVAL, "sn create: boundary edge off the box");

    // ---- dependency levels per direction (Kahn), classification in FP64
    std::vector<int> level((size_t)nd * T, 0);
    std::vector<int> nlev(nd, 0);
    // inflow / outflow by the sign of Omega . n, taken with the azimuth's unit in-plane
    // vector so that the P polar directions of one azimuth (the same vector scaled by
    // sin(theta_p)) always agree, also for faces almost parallel to it
    std::vector<double> azc(A), azs(A);
    for (int a = 0; a < A; ++a) {
        const double ph = 2.0 * 3.14159265358979323846 * (a + 0.5) / A;
        azc[a] = std::cos(ph);
        azs[a] = std::sin(ph);
    }
    auto onf = [&](int dd, int e, int k) {
        const int a = dd / P;
        return azc[a] * nrm[((size_t)e * 3 + k) * 2] + azs[a] * nrm[((size_t)e * 3 + k) * 2 + 1];
    };
    parallel_for(nd, c->n_threads, 1, [&](int64_t d0, int64_t d1, int) {
        std::vector<int> indeg(T), queue(T);
        for (int64_t dd = d0; dd < d1; ++dd) {
            int *lev = &level[(size_t)dd * T];
            for (int e = 0; e < T; ++e) {
                indeg[e] = 0;
                for (int k = 0; k < 3; ++k)
                    if (nbr[(size_t)e * 3 + k] >= 0 && onf((int)dd, e, k) < 0) ++indeg[e];
            }
            int head = 0, tail = 0;
            for (int e = 0; e < T; ++e)
                if (indeg[e] == 0) queue[tail++] = e;
            while (head < tail) {
                const int e = queue[head++];
                for (int k = 0; k < 3; ++k) {
                    const int nb = nbr[(size_t)e * 3 + k];
                    if (nb >= 0 && onf((int)dd, e, k) > 0) {
                        lev[nb] = std::max(lev[nb], lev[e] + 1);
                        if (--indeg[nb] == 0) queue[tail++] = nb;
                    }
                }
            }
            if (tail != T) throw Error(MOC_EINVAL, "sn create: cyclic sweep dependencies");
            int mx = 0;
            for (int e = 0; e < T; ++e) mx = std::max(mx, lev[e]);
            nlev[dd] = mx + 1;
        }
    });
    int nsteps = 0;
    for (int v : nlev) nsteps = std::max(nsteps, v);
    d.nsteps = nsteps;

    // ---- tasks ordered by level, then element, then direction
    const int64_t ntask = (int64_t)nd * T;
    d.ntask = ntask;
    d.step_off.assign(nsteps + 1, 0);
    for (int64_t i = 0; i < ntask; ++i) ++d.step_off[level[i] + 1];
    for (int s = 0; s < nsteps; ++s) d.step_off[s + 1] += d.step_off[s];
    std::vector<int64_t> fillp(d.step_off.begin(), d.step_off.end() - 1);
    std::vector<int> task_e(ntask), task_d(ntask);
    std::vector<int64_t> task_of((size_t)ntask);   // (direction, element) -> task
    for (int e = 0; e < T; ++e)
        for (int dd = 0; dd < nd; ++dd) {
            const int64_t k = fillp[level[(size_t)dd * T + e]]++;
            task_e[k] = e;
            task_d[k] = dd;
            task_of[(size_t)dd * T + e] = k;
        }

    // ---- the P polar directions of one azimuth see the same in-plane upwind structure, so
    // an (element, azimuth) normally has its P tasks side by side in one level; the sweep
    // step then takes them in one thread (one scalar-flux update instead of P). Any level
    // that breaks the pattern (a face almost parallel to a direction can round differently
    // for different polar angles) makes every step take one task per thread.
    {
        int tg = P;
        for (int s2 = 0; s2 < nsteps && tg > 1; ++s2) {
            const int64_t k0 = d.step_off[s2], k1 = d.step_off[s2 + 1];
            if ((k1 - k0) % P) {
                tg = 1;
                break;
            }
            for (int64_t k = k0; k < k1 && tg > 1; k += P)
                for (int p = 0; p < P; ++p)
                    if (task_e[k + p] != task_e[k] || task_d[k + p] != task_d[k] + p || task_d[k] % P != 0) {
                        tg = 1;
                        break;
                    }
        }
        d.tgroup = tg;
    }

    // ---- compressed storage (Alg. DFEM_SN_sweep): a task's slot is held until the last
    // downstream element that reads it has been swept, then reused
    std::vector<int> last_use(ntask);
    for (int64_t k = 0; k < ntask; ++k) {
        const int e = task_e[k], dd = task_d[k];
        int lu = level[(size_t)dd * T + e];
        for (int f = 0; f < 3; ++f) {
            const int nb = nbr[(size_t)e * 3 + f];
            if (nb >= 0 && onf(dd, e, f) > 0) lu = std::max(lu, level[(size_t)dd * T + nb]);
        }
        last_use[k] = lu;
    }
    std::vector<int> slot(ntask, -1), free_slots;
    std::vector<std::vector<int>> release(nsteps);
    int next_slot = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (s > 0)
            for (int sl : release[s - 1]) free_slots.push_back(sl);
        for (int64_t k = d.step_off[s]; k < d.step_off[s + 1]; ++k) {
            int sl;
            if (!free_slots.empty()) {
                sl = free_slots.back();
                free_slots.pop_back();
            } else {
                sl = next_slot++;
            }
            slot[k] = sl;
            release[last_use[k]].push_back(sl);
        }
    }
    d.nslot = next_slot;

    // ---- boundary faces and the inflow code of every (task, face)
    std::vector<int> bface(3 * (size_t)T, -1);
    int64_t nbf = 0;
    for (int h = 0; h < 3 * T; ++h)
        if (m.twin[h] < 0) bface[h] = (int)nbf++;
    d.nbnd = nbf * nd;
    std::vector<int> inflow(3 * (size_t)ntask), bwrite(3 * (size_t)ntask, -1);
    for (int64_t k = 0; k < ntask; ++k) {
        const int e = task_e[k], dd = task_d[k];
        for (int f = 0; f < 3; ++f) {
            const int nb = nbr[(size_t)e * 3 + f];
            const double on = onf(dd, e, f);
            int code = kSnOutflow;
            if (nb >= 0) {
                if (on < 0) code = slot[task_of[(size_t)dd * T + nb]];
            } else {
                const int side = -1 - nb;
                const bool refl = m.bc[side] == MOC_BC_REFLECTIVE;
                const int bf = bface[3 * e + f];
                if (on < 0) {
                    code = refl ? -4 - (bf * nd + (side < 2 ? rx[dd] : ry[dd])) : kSnVacuum;
                } else if (refl) {
                    bwrite[3 * k + f] = bf * nd + dd;
                }
            }
            inflow[3 * k + f] = code;
        }
    }

    {
        SnHost &h = c->h;
        h.T = T;
        h.A = A;
        h.P = P;
        h.nd = nd;
        h.nbr = nbr;
        h.nrm = nrm;
        h.azc = azc;
        h.azs = azs;
        h.bface = bface;
        h.rx = rx;
        h.ry = ry;
        for (int i = 0; i < 6; ++i) h.bc[i] = m.bc[i];
    }
    d.ndg = nd / d.tgroup;

    // ---- check the schedule on the host before any kernel can use it: replay the sweep
    // order and require every upstream read to find its task's flux in the slot, and every
    // index to be in range
    {
        std::vector<int64_t> owner(std::max<int64_t>(d.nslot, 1), -1);
        for (int st2 = 0; st2 < nsteps; ++st2) {
            for (int64_t k = d.step_off[st2]; k < d.step_off[st2 + 1]; ++k) {
                const int e = task_e[k], dd = task_d[k];
                for (int f = 0; f < 3; ++f) {
                    const int code = inflow[3 * k + f];
                    if (code >= 0) {
                        const int nb = nbr[(size_t)e * 3 + f];
                        if (code >= d.nslot || nb < 0 || owner[code] != task_of[(size_t)dd * T + nb])
                            throw Error(MOC_EINVAL, "sn create: inconsistent angular-flux storage schedule");
                    } else if (code <= -4) {
                        if (-4 - (int64_t)code >= d.nbnd) throw Error(MOC_EINVAL, "sn create: boundary index out of range");
                    } else if (code != kSnOutflow && code != kSnVacuum) {
                        throw Error(MOC_EINVAL, "sn create: bad inflow code");
                    }
                    if (bwrite[3 * k + f] >= d.nbnd) throw Error(MOC_EINVAL, "sn create: boundary index out of range");
                }
            }
            for (int64_t k = d.step_off[st2]; k < d.step_off[st2 + 1]; ++k) {
                if (slot[k] < 0 || slot[k] >= d.nslot) throw Error(MOC_EINVAL, "sn create: slot out of range");
                owner[slot[k]] = k;
            }
        }
    }
    if (o.device < 0) {
        c->host_only = true;
        c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return;
    }

    // ---- device
    c->device = o.device;
    SN_HIP(hipSetDevice(c->device));
    SN_HIP(hipStreamCreate(&c->stream));
    SN_HIP(hipHostMalloc((void **)&c->host_scal, kSnCount * sizeof(double)));
    auto up_real = [&](const std::vector<double> &v) -> void * {
        if (f64) return c->upload(v);
        return c->upload(std::vector<float>(v.begin(), v.end()));
    };
    std::vector<int> mat(T);
    for (int e = 0; e < T; ++e) mat[e] = mesh_in->region_material[m.tri_region[e]];
    // Sigma_t per (element, group), so the sweep step reads it without the material hop
    std::vector<double> st((size_t)T * G);
    for (int e = 0; e < T; ++e)
        for (int g = 0; g < G; ++g) st[(size_t)e * G + g] = xs->sigma_t[(size_t)mat[e] * G + g];
    d.mass = up_real(mass);
    d.fmass = up_real(fmass);
    d.fcpl = up_real(fcpl);
    d.nrm = up_real(nrm);
    d.gradw = up_real(gradw);
    d.sigt = up_real(st);
    d.dirs = up_real(dirs);
    d.area = c->upload(area);
    d.massd = c->upload(mass9);
    d.mat = c->upload(mat);
    d.sigs_m = c->upload(std::vector<double>(xs->sigma_s, xs->sigma_s + (size_t)M * G * G));
    d.nsf_m = c->upload(std::vector<double>(xs->nu_sigma_f, xs->nu_sigma_f + M * G));
    d.chi_m = c->upload(std::vector<double>(xs->chi, xs->chi + M * G));
    d.task_e = c->upload(task_e);
    d.task_d = c->upload(task_d);
    d.task_slot = c->upload(slot);
    d.inflow = c->upload(inflow);
    d.bwrite = c->upload(bwrite);
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    d.psi = c->dalloc<char>((size_t)std::max<int64_t>(d.nslot, 1) * G * 3 * rs);
    d.bnd[0] = c->dalloc<char>((size_t)std::max<int64_t>(d.nbnd, 1) * G * 3 * rs);
    d.bnd[1] = c->dalloc<char>((size_t)std::max<int64_t>(d.nbnd, 1) * G * 3 * rs);
    d.q = c->dalloc<char>((size_t)T * G * 3 * rs);
    d.phi_acc = c->dalloc<double>((size_t)T * G * 3);
    // scalar-flux contribution of each (element, direction group), gathered in direction order
    d.run_acc = f64 ? (void *)c->dalloc<double>((size_t)T * d.ndg * G * 3) : (void *)c->dalloc<float>((size_t)T * d.ndg * G * 3);
    d.phi[0] = c->dalloc<double>((size_t)T * G * 3);
    d.phi[1] = c->dalloc<double>((size_t)T * G * 3);
    d.partials = c->dalloc<double>(2 * kSnReduceBlocks);
    d.scal = c->dalloc<double>(kSnCount);
    hipStream_t s = c->stream;
    launch_sn_fill(d.bnd[0], d.nbnd * G * 3, d.precision, s);
    launch_sn_fill(d.bnd[1], d.nbnd * G * 3, d.precision, s);
    launch_sn_fill(d.q, (int64_t)T * G * 3, d.precision, s);
    launch_sn_cold(d.phi[0], (int64_t)T * G * 3, s);
    launch_sn_fill_f64(d.scal, kSnCount, 0.0, s);
    launch_sn_fill_f64(d.scal + kSnK, 1, 1.0, s);
    SN_HIP(hipStreamSynchronize(s));
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static std::pair<hipEvent_t, hipEvent_t> sn_prof_events(moc_sn_ctx *c) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->prof_pool.empty()) {
        SN_HIP(hipEventCreate(&ev.first));
        SN_HIP(hipEventCreate(&ev.second));
    } else {
        ev = c->prof_pool.back();
        c->prof_pool.pop_back();
    }
    return ev;
}

// The launches of one sweep with the emission in d.q: one launch per dependency level
// (every direction's elements of that level, all groups), or with tiles one launch per
// tile level, then the gather of the scalar flux; reflective inflow reads boundary buffer
// `parity`, outflow writes the other.
static void sn_enqueue_sweep(moc_sn_ctx *c, int parity, hipStream_t s) {
    DevSN &d = c->d;
    SnStepArgs a{};
    a.mass = d.mass;
    a.fmass = d.fmass;
    a.fcpl = d.fcpl;
    a.nrm = d.nrm;
    a.gradw = d.gradw;
    a.sigt = d.sigt;
    a.dirs = d.dirs;
    a.q = d.q;
    a.mat = d.mat;
    a.task_e = d.task_e;
    a.task_d = d.task_d;
    a.task_slot = d.task_slot;
    a.inflow = d.inflow;
    a.bwrite = d.bwrite;
    a.psi = d.psi;
    a.bnd_in = d.bnd[parity];
    a.bnd_out = d.bnd[1 - parity];
    a.run_acc = d.run_acc;
    a.G = d.G;
    a.tgroup = d.tgroup;
    a.ndg = d.ndg;
    a.T = d.T;
    if (c->tiled) {
        const DevSNTiles &t = c->tl;
        a.psi = t.psi;
        SnTileArgs ta{};
        ta.tt_task = t.tt_task;
        ta.tt_fine = t.tt_fine;
        ta.fine_off = t.fine_off;
        ta.tt_tile = t.tt_tile;
        ta.tt_dg = t.tt_dg;
        ta.tile_off = t.tile_off;
        ta.tile_elems = t.tile_elems;
        ta.ext_off = t.ext_off;
        ta.ext_src = t.ext_src;
        ta.rec = t.rec;
        for (int r = 0; r < kSnLdsCount; ++r) ta.lds_off[r] = t.lds_off[r];
        ta.el_stride = t.el_stride;
        for (int L = 0; L < t.n_levels; ++L) {
            ta.tt0 = t.lev_off[L];
            launch_sn_tile(a, ta, (int)(t.lev_off[L + 1] - t.lev_off[L]), t.lds_bytes, d.precision, s);
        }
    } else {
        for (int st = 0; st < d.nsteps; ++st) {
            a.k0 = d.step_off[st];
            a.k1 = d.step_off[st + 1];
            launch_sn_step(a, d.precision, s);
        }
    }
    launch_sn_gather(d, s);
}

// One sweep. The hundreds of small per-level launches and the final gather are recorded
// once per parity into a HIP graph (kernel nodes only) and replayed, which removes most of
// the per-launch cost.
static void sn_sweep_impl(moc_sn_ctx *c, hipStream_t s) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    const int parity = c->cur_bnd;
    if (!c->graph[parity]) {
        hipGraph_t g = nullptr;
        SN_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        try {
            sn_enqueue_sweep(c, parity, c->stream);
        } catch (...) {
            (void)hipStreamEndCapture(c->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        SN_HIP(hipStreamEndCapture(c->stream, &g));
        const hipError_t ie = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) throw Error(MOC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    if (c->profiling) {
        ev = sn_prof_events(c);
        SN_HIP(hipEventRecord(ev.first, s));
    }
    SN_HIP(hipGraphLaunch(c->graph[parity], s));
    c->cur_bnd = 1 - c->cur_bnd;
    if (c->profiling) {
        SN_HIP(hipEventRecord(ev.second, s));
        c->prof_pending.push_back(ev);
    }
}

// LDS of one block of the tiled sweep when no device is there to ask (host-only contexts):
// gfx950's 160 KiB
constexpr size_t kSnHostLdsLimit = 160 * 1024;

static void sn_drop_graphs(moc_sn_ctx *c) {
    if (c->stream) SN_HIP(hipStreamSynchronize(c->stream));
    for (auto &g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

static void sn_clear_tiles(moc_sn_ctx *c) {
    sn_drop_graphs(c);
    for (void *p : c->tile_allocs) c->dfree(p);
    c->tile_allocs.clear();
    c->tl = DevSNTiles{};
    c->tiled = false;
}

// The tiled schedule (an MI355X layout of the same dependency order, Alg. DFEM_SN_sweep):
// per direction group, the tiles' own dependency graph (a tile feeds another through the
// faces between them) ordered by Kahn's algorithm into tile levels, and inside each tile
// the elements' levels restricted to the tile. One tile level is one launch; a tile task
// (tile, direction group) is one block that walks its inner levels. Fluxes read inside a
// tile stay in LDS; fluxes read by another tile get a storage slot, allocated over tile
// levels as the level schedule allocates them over levels. Everything is checked by a
// host replay before any upload.
static void sn_set_tiles_impl(moc_sn_ctx *c, int n_tiles, const int32_t *tile_of) {
    if (n_tiles <= 0 || !tile_of) {
        if (n_tiles > 0 || tile_of) throw Error(MOC_EINVAL, "sn tiles: n_tiles > 0 needs element_tile and back");
        sn_clear_tiles(c);
        return;
    }
    const SnHost &h = c->h;
    const DevSN &d = c->d;
    const int T = h.T, nd = h.nd, TG = d.tgroup, ndg = d.ndg, G = d.G;
    const bool f64 = d.precision == MOC_PREC_F64;
    // tiles and each element's index within its tile
    std::vector<int> tsize(n_tiles, 0), local(T);
    for (int e = 0; e < T; ++e) {
        const int t = tile_of[e];
        if (t < 0 || t >= n_tiles) throw Error(MOC_EINVAL, "sn tiles: tile index out of range");
        local[e] = tsize[t]++;
    }
    int max_tile = 0;
    for (int t = 0; t < n_tiles; ++t) {
        if (tsize[t] == 0) throw Error(MOC_EINVAL, "sn tiles: empty tile " + std::to_string(t));
        max_tile = std::max(max_tile, tsize[t]);
    }
    size_t lds_limit = kSnHostLdsLimit;
    if (!c->host_only) {
        int v = 0;
        SN_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
        lds_limit = (size_t)v;
    }
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    std::vector<int> toff(n_tiles + 1, 0), telem(T);
    for (int t = 0; t < n_tiles; ++t) toff[t + 1] = toff[t] + tsize[t];
    {
        std::vector<int> fill(toff.begin(), toff.end() - 1);
        for (int e = 0; e < T; ++e) telem[fill[tile_of[e]]++] = e;   // ascending element order
    }
    // per direction group: tile levels and the elements' levels inside their tile
    std::vector<int> tlev((size_t)ndg * n_tiles), flev((size_t)ndg * T);
    std::vector<int> ntlev(ndg, 0);
    parallel_for(ndg, c->n_threads, 1, [&](int64_t g0, int64_t g1, int) {
        std::vector<int> indeg(std::max(T, n_tiles)), queue(std::max(T, n_tiles));
        for (int64_t dg = g0; dg < g1; ++dg) {
            const int dd = (int)dg * TG;
            int *tl = &tlev[(size_t)dg * n_tiles];
            // tile graph: one edge per face from one tile into another
            std::fill(indeg.begin(), indeg.begin() + n_tiles, 0);
            for (int e = 0; e < T; ++e)
                for (int k = 0; k < 3; ++k) {
                    const int nb = h.nbr[(size_t)e * 3 + k];
                    if (nb >= 0 && tile_of[nb] != tile_of[e] && h.onf(dd, e, k) > 0) ++indeg[tile_of[nb]];
                }
            int head = 0, tail = 0;
            for (int t = 0; t < n_tiles; ++t) {
                tl[t] = 0;
                if (indeg[t] == 0) queue[tail++] = t;
            }
            while (head < tail) {
                const int t = queue[head++];
                for (int i = toff[t]; i < toff[t + 1]; ++i) {
                    const int e = telem[i];
                    for (int k = 0; k < 3; ++k) {
                        const int nb = h.nbr[(size_t)e * 3 + k];
                        if (nb >= 0 && tile_of[nb] != t && h.onf(dd, e, k) > 0) {
                            const int tn = tile_of[nb];
                            tl[tn] = std::max(tl[tn], tl[t] + 1);
                            if (--indeg[tn] == 0) queue[tail++] = tn;
                        }
                    }
                }
            }
            if (tail != n_tiles)
                throw Error(MOC_EINVAL, "sn tiles: the tiles' sweep dependencies are cyclic for direction " +
                                            std::to_string(dd) + " (use convex tiles)");
            int mx = 0;
            for (int t = 0; t < n_tiles; ++t) mx = std::max(mx, tl[t]);
            ntlev[dg] = mx + 1;
            // levels inside each tile (edges between elements of the same tile)
            int *fl = &flev[(size_t)dg * T];
            for (int e = 0; e < T; ++e) {
                fl[e] = 0;
                indeg[e] = 0;
                for (int k = 0; k < 3; ++k) {
                    const int nb = h.nbr[(size_t)e * 3 + k];
                    if (nb >= 0 && tile_of[nb] == tile_of[e] && h.onf(dd, e, k) < 0) ++indeg[e];
                }
            }
            head = tail = 0;
            for (int e = 0; e < T; ++e)
                if (indeg[e] == 0) queue[tail++] = e;
            while (head < tail) {
                const int e = queue[head++];
                for (int k = 0; k < 3; ++k) {
                    const int nb = h.nbr[(size_t)e * 3 + k];
                    if (nb >= 0 && tile_of[nb] == tile_of[e] && h.onf(dd, e, k) > 0) {
                        fl[nb] = std::max(fl[nb], fl[e] + 1);
                        if (--indeg[nb] == 0) queue[tail++] = nb;
                    }
                }
            }
            if (tail != T) throw Error(MOC_EINVAL, "sn tiles: cyclic dependencies inside a tile");
        }
    });
    int nlev = 0;
    for (int v : ntlev) nlev = std::max(nlev, v);

    // tile tasks ordered by (tile level, direction group, tile); inside a tile task the
    // tasks by (inner level, element, direction)
    DevSNTiles tl;
    tl.n_tiles = n_tiles;
    tl.n_levels = nlev;
    tl.max_tile = max_tile;
    const int64_t ntt = (int64_t)ndg * n_tiles, ntask = (int64_t)T * nd;
    tl.lev_off.assign(nlev + 1, 0);
    for (int64_t dg = 0; dg < ndg; ++dg)
        for (int t = 0; t < n_tiles; ++t) ++tl.lev_off[tlev[(size_t)dg * n_tiles + t] + 1];
    for (int L = 0; L < nlev; ++L) tl.lev_off[L + 1] += tl.lev_off[L];
    std::vector<int64_t> tt_order(ntt);
    {
        std::vector<int64_t> fill(tl.lev_off.begin(), tl.lev_off.end() - 1);
        for (int64_t dg = 0; dg < ndg; ++dg)
            for (int t = 0; t < n_tiles; ++t) tt_order[fill[tlev[(size_t)dg * n_tiles + t]]++] = dg * n_tiles + t;
    }
    std::vector<int> task_e(ntask), task_d(ntask), task_loc(ntask), tt_fine(ntt + 1), tt_tile(ntt), tt_dg(ntt);
    std::vector<int64_t> tt_task(ntt + 1), task_of(ntask), task_tt(ntask);
    std::vector<int> task_fl(ntask), fine_off;
    fine_off.reserve((size_t)ntt * 8);
    int64_t k = 0;
    std::vector<int> order;
    for (int64_t i = 0; i < ntt; ++i) {
        const int64_t dg = tt_order[i] / n_tiles;
        const int t = (int)(tt_order[i] % n_tiles);
        const int *fl = &flev[(size_t)dg * T];
        order.assign(telem.begin() + toff[t], telem.begin() + toff[t + 1]);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return fl[x] < fl[y]; });
        tt_task[i] = k;
        tt_fine[i] = (int)fine_off.size();
        tt_tile[i] = t;
        tt_dg[i] = (int)dg;
        int cur = -1;
        for (int e : order) {
            if (fl[e] != cur) {
                cur = fl[e];
                fine_off.push_back((int)(k - tt_task[i]));
            }
            for (int p = 0; p < TG; ++p) {
                const int dd = (int)dg * TG + p;
                task_e[k] = e;
                task_d[k] = dd;
                task_loc[k] = local[e];
                task_of[(size_t)dd * T + e] = k;
                task_tt[k] = i;
                task_fl[k] = cur;
                ++k;
            }
        }
        fine_off.push_back((int)(k - tt_task[i]));
    }
    tt_task[ntt] = k;
    tt_fine[ntt] = (int)fine_off.size();
    if (k != ntask) throw Error(MOC_EINVAL, "sn tiles: task count mismatch");
    std::vector<int> tt_level(ntt);
    for (int L = 0; L < nlev; ++L)
        for (int64_t i = tl.lev_off[L]; i < tl.lev_off[L + 1]; ++i) tt_level[i] = L;

    // items: (tile task, element); task k belongs to item k / TG as polar direction k % TG
    const int64_t nitem = ntask / TG;
    auto bad = [](const char *what) { throw Error(MOC_EINVAL, std::string("sn tiles: inconsistent schedule (") + what + ")"); };
    // storage slots for fluxes read by another tile, TG consecutive slots per item (one per
    // polar direction): held from the producing tile level to the last reading one, then
    // reused
    std::vector<int> last_use(nitem, -1);
    for (int64_t it = 0; it < nitem; ++it) {
        const int e = task_e[it * TG], dd = task_d[it * TG];
        for (int f = 0; f < 3; ++f) {
            const int nb = h.nbr[(size_t)e * 3 + f];
            if (nb >= 0 && tile_of[nb] != tile_of[e] && h.onf(dd, e, f) > 0)
                last_use[it] = std::max(last_use[it], tt_level[task_tt[task_of[(size_t)dd * T + nb]]]);
        }
    }
    std::vector<int> sgrp(nitem, -1), free_slots;
    {
        std::vector<std::vector<int>> release(nlev);
        int next = 0;
        for (int L = 0; L < nlev; ++L) {
            if (L > 0)
                for (int sl : release[L - 1]) free_slots.push_back(sl);
            for (int64_t it = tt_task[tl.lev_off[L]] / TG; it < tt_task[tl.lev_off[L + 1]] / TG; ++it) {
                if (last_use[it] < 0) continue;
                int sl;
                if (!free_slots.empty()) {
                    sl = free_slots.back();
                    free_slots.pop_back();
                } else {
                    sl = next++;
                }
                sgrp[it] = sl;
                release[last_use[it]].push_back(sl);
            }
        }
        tl.nslot = (int64_t)next * TG;
    }
    if (tl.nslot >= kSnExtFlag) throw Error(MOC_EINVAL, "sn tiles: too many storage slots");
    auto slot_of = [&](int64_t kk) { return sgrp[kk / TG] >= 0 ? sgrp[kk / TG] * TG + (int)(kk % TG) : -1; };
    // LDS slots inside each tile task (Alg. DFEM_SN_sweep's compressed storage within the
    // tile): an element's fluxes are held from its inner level to the last inner level that
    // reads them
    std::vector<int> lslot(nitem, -1);
    int max_live = 1;
    {
        std::vector<int> lu(nitem, -1), freel;
        std::vector<std::vector<int>> rel;
        for (int64_t i = 0; i < ntt; ++i) {
            const int nf = tt_fine[i + 1] - tt_fine[i] - 1;
            for (int64_t it = tt_task[i] / TG; it < tt_task[i + 1] / TG; ++it) {
                const int e = task_e[it * TG], dd = task_d[it * TG];
                for (int f = 0; f < 3; ++f) {
                    const int nb = h.nbr[(size_t)e * 3 + f];
                    if (nb >= 0 && tile_of[nb] == tile_of[e] && h.onf(dd, e, f) > 0)
                        lu[it] = std::max(lu[it], task_fl[task_of[(size_t)dd * T + nb]]);
                }
            }
            rel.assign(nf + 1, {});
            freel.clear();
            int next = 0;
            for (int j = 0; j < nf; ++j) {
                if (j > 0)
                    for (int sl : rel[j - 1]) freel.push_back(sl);
                const int64_t ia = (tt_task[i] + fine_off[tt_fine[i] + j]) / TG, ib = (tt_task[i] + fine_off[tt_fine[i] + j + 1]) / TG;
                for (int64_t it = ia; it < ib; ++it) {
                    if (lu[it] < 0) continue;
                    if (lu[it] <= j || lu[it] >= nf) bad("inner reader level");
                    int sl;
                    if (!freel.empty()) {
                        sl = freel.back();
                        freel.pop_back();
                    } else {
                        sl = next++;
                    }
                    lslot[it] = sl;
                    rel[lu[it]].push_back(sl);
                }
            }
            max_live = std::max(max_live, next);
        }
    }

    // inflow codes and boundary writes of every task
    std::vector<int> inflow(3 * (size_t)ntask), bwrite(3 * (size_t)ntask, -1);
    for (int64_t kk = 0; kk < ntask; ++kk) {
        const int e = task_e[kk], dd = task_d[kk];
        for (int f = 0; f < 3; ++f) {
            const int nb = h.nbr[(size_t)e * 3 + f];
            const double on = h.onf(dd, e, f);
            int code = kSnOutflow;
            if (nb >= 0) {
                if (on < 0) {
                    const int64_t kp = task_of[(size_t)dd * T + nb];
                    code = tile_of[nb] == tile_of[e] ? (kSnLocalFlag | lslot[kp / TG]) : slot_of(kp);
                }
            } else {
                const int side = -1 - nb;
                const bool refl = h.bc[side] == MOC_BC_REFLECTIVE;
                const int bf = h.bface[3 * e + f];
                if (on < 0) {
                    code = refl ? -4 - (bf * nd + (side < 2 ? h.rx[dd] : h.ry[dd])) : kSnVacuum;
                } else if (refl) {
                    bwrite[3 * kk + f] = bf * nd + dd;
                }
            }
            inflow[3 * kk + f] = code;
        }
    }

    // replay: every read finds its producer's flux (a storage slot written at an earlier
    // tile level and not rewritten since; an LDS slot of the same tile task written at an
    // earlier inner level and not rewritten since), no storage slot is written at the tile
    // level that reads its previous value, and every index is in range
    {
        std::vector<int64_t> owner(std::max<int64_t>(tl.nslot, 1), -1);
        std::vector<int> last_read(std::max<int64_t>(tl.nslot, 1), -1), written(std::max<int64_t>(tl.nslot, 1), -1);
        std::vector<int64_t> lowner(max_live, -1);
        for (int L = 0; L < nlev; ++L) {
            for (int64_t i = tl.lev_off[L]; i < tl.lev_off[L + 1]; ++i) {
                std::fill(lowner.begin(), lowner.end(), -1);
                for (int j = tt_fine[i]; j < tt_fine[i + 1] - 1; ++j) {
                    const int64_t ka = tt_task[i] + fine_off[j], kb = tt_task[i] + fine_off[j + 1];
                    for (int64_t kk = ka; kk < kb; ++kk) {
                        const int e = task_e[kk], dd = task_d[kk];
                        if (task_loc[kk] < 0 || task_loc[kk] >= max_tile) bad("tile index");
                        for (int f = 0; f < 3; ++f) {
                            const int code = inflow[3 * kk + f];
                            const int nb = h.nbr[(size_t)e * 3 + f];
                            if (code >= 0 && (code & kSnLocalFlag)) {
                                const int ls = code & ~kSnLocalFlag;
                                if (nb < 0 || tile_of[nb] != tile_of[e] || ls >= max_live) bad("local read");
                                const int64_t kp = task_of[(size_t)dd * T + nb];
                                if (lowner[ls] != kp / TG || task_tt[kp] != i || task_fl[kp] >= task_fl[kk]) bad("local read order");
                            } else if (code >= 0) {
                                if (code >= tl.nslot || nb < 0 || owner[code] != task_of[(size_t)dd * T + nb]) bad("slot read");
                                last_read[code] = L;
                            } else if (code <= -4) {
                                if (-4 - (int64_t)code >= d.nbnd) bad("boundary index");
                            } else if (code != kSnOutflow && code != kSnVacuum) {
                                bad("inflow code");
                            }
                            if (bwrite[3 * kk + f] >= d.nbnd) bad("boundary index");
                        }
                    }
                    for (int64_t it = ka / TG; it < kb / TG; ++it)
                        if (lslot[it] >= 0) lowner[lslot[it]] = it;
                }
            }
            for (int64_t kk = tt_task[tl.lev_off[L]]; kk < tt_task[tl.lev_off[L + 1]]; ++kk) {
                const int sl = slot_of(kk);
                if (sl < 0) continue;
                if (sl >= tl.nslot || written[sl] == L || last_read[sl] >= L) bad("slot write");
                written[sl] = L;
                owner[sl] = kk;
            }
        }
        for (int64_t i = 0; i < ntt; ++i) {
            const int n_fine = tt_fine[i + 1] - tt_fine[i] - 1;
            if (n_fine < 1) bad("empty tile task");
            if (tt_task[i] + fine_off[tt_fine[i + 1] - 1] != tt_task[i + 1] || tt_task[i] % TG) bad("tile task extent");
            for (int j = tt_fine[i]; j < tt_fine[i + 1] - 1; ++j)
                if (fine_off[j + 1] <= fine_off[j] || (fine_off[j + 1] - fine_off[j]) % TG) bad("inner level");
        }
    }

    // item records [tile element, LDS slot, three inflow codes, three boundary writes,
    // storage slot], written for polar direction 0; direction p of the item adds p to a
    // staged entry (kSnExtFlag | j), subtracts it from a reflective code (-4 - j), and adds
    // it to a boundary write and to the storage slot. Every flux a tile task reads from a
    // storage slot or the boundary buffer becomes a staged entry, TG consecutive ones per
    // (item, face).
    std::vector<int> rec((size_t)nitem * kSnRecInts), ext_off(ntt + 1, 0), ext_src;
    int max_ext = 0, max_fine = 0, max_items = 0;
    for (int64_t i = 0; i < ntt; ++i) {
        ext_off[i] = (int)ext_src.size();
        for (int64_t it = tt_task[i] / TG; it < tt_task[i + 1] / TG; ++it) {
            int *r = &rec[(size_t)it * kSnRecInts];
            const int64_t k0 = it * TG;
            r[0] = task_loc[k0];
            r[1] = lslot[it];
            for (int f = 0; f < 3; ++f) {
                const int c0 = inflow[3 * k0 + f];
                const bool staged = (c0 >= 0 && !(c0 & kSnLocalFlag)) || c0 <= -4;
                int code = c0;
                if (staged) {
                    const int j = (int)ext_src.size() - ext_off[i];
                    if (j + TG >= kSnExtFlag) throw Error(MOC_EINVAL, "sn tiles: too many inflow entries in one tile");
                    for (int p = 0; p < TG; ++p) ext_src.push_back(inflow[3 * (k0 + p) + f]);
                    code = c0 >= 0 ? (kSnExtFlag | j) : -4 - j;
                }
                r[2 + f] = code;
                r[5 + f] = bwrite[3 * k0 + f];
                // every polar direction of the item must follow from direction 0's record
                for (int p = 0; p < TG; ++p) {
                    const int cp = inflow[3 * (k0 + p) + f], bw = bwrite[3 * (k0 + p) + f];
                    if (staged) {
                        const int jp = (c0 >= 0 ? (code & ~kSnExtFlag) : -4 - code) + p;
                        if (((cp >= 0) != (c0 >= 0)) || ext_src[ext_off[i] + jp] != cp) bad("staged entry");
                    } else if (cp != c0) {
                        bad("polar inflow code");
                    }
                    if ((bw >= 0) != (r[5 + f] >= 0) || (bw >= 0 && bw != r[5 + f] + p)) bad("polar boundary write");
                }
            }
            r[8] = slot_of(k0);
            for (int p = 0; p < TG; ++p)
                if (slot_of(k0 + p) != (r[8] >= 0 ? r[8] + p : -1) || task_loc[k0 + p] != r[0]) bad("polar slot");
        }
        max_ext = std::max(max_ext, (int)ext_src.size() - ext_off[i]);
        max_fine = std::max(max_fine, tt_fine[i + 1] - tt_fine[i]);
        max_items = std::max(max_items, (int)((tt_task[i + 1] - tt_task[i]) / TG));
        tl.max_inner = std::max(tl.max_inner, tt_fine[i + 1] - tt_fine[i] - 1);
    }
    ext_off[ntt] = (int)ext_src.size();
    tl.max_live = max_live;
    // staged element data per item: the head and, per face, the matrix its direction group
    // uses (coupling matrix for an interior inflow, face matrix for an outflow or a
    // reflective inflow, nothing for a vacuum inflow)
    int el_stride = kSnElemHead;
    for (int64_t it = 0; it < nitem; ++it) {
        int n = kSnElemHead;
        for (int f = 0; f < 3; ++f) {
            const int c = rec[(size_t)it * kSnRecInts + 2 + f];
            n += c == kSnVacuum ? 0 : (c >= 0 ? 9 : 6);
        }
        el_stride = std::max(el_stride, n);
    }
    tl.el_stride = el_stride;
    // LDS layout of one block (16-byte aligned regions)
    {
        const size_t sz[kSnLdsCount] = {(size_t)max_live * TG * G * 3 * rs, (size_t)max_items * el_stride * rs,
                                        (size_t)max_tile * G * 4 * rs,      (size_t)max_ext * G * 3 * rs,
                                        (size_t)TG * 3 * rs,                (size_t)max_items * kSnRecInts * sizeof(int),
                                        (size_t)max_tile * sizeof(int),     (size_t)max_fine * sizeof(int)};
        size_t off = 0;
        for (int r = 0; r < kSnLdsCount; ++r) {
            tl.lds_off[r] = (unsigned)off;
            off += (sz[r] + 15) & ~(size_t)15;
        }
        tl.lds_bytes = off;
        if (off > lds_limit)
            throw Error(MOC_EINVAL, "sn tiles: a tile of " + std::to_string(max_tile) + " elements needs " + std::to_string(off) +
                                        " bytes of LDS (the device allows " + std::to_string(lds_limit) + ")");
    }

    sn_clear_tiles(c);
    if (!c->host_only) {
        SN_HIP(hipSetDevice(c->device));
        auto up = [&](const auto &v) {
            auto *p = c->upload(v);
            c->tile_allocs.push_back(p);
            return p;
        };
        tl.rec = up(rec);
        tl.tt_task = up(tt_task);
        tl.tt_fine = up(tt_fine);
        tl.fine_off = up(fine_off);
        tl.tt_tile = up(tt_tile);
        tl.tt_dg = up(tt_dg);
        tl.tile_off = up(toff);
        tl.tile_elems = up(telem);
        tl.ext_off = up(ext_off);
        tl.ext_src = up(ext_src.empty() ? std::vector<int>(1, 0) : ext_src);
        tl.psi = c->dalloc<char>((size_t)std::max<int64_t>(tl.nslot, 1) * G * 3 * rs);
        c->tile_allocs.push_back(tl.psi);
    }
    c->tl = std::move(tl);
    c->tiled = true;
}

static void sn_drain_profile(moc_sn_ctx *c) {
    for (auto &e : c->prof_pending) {
        SN_HIP(hipEventSynchronize(e.second));
        float ms = 0;
        SN_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_ms += ms;
        c->prof_min = c->prof_n == 0 ? ms : std::min(c->prof_min, (double)ms);
        c->prof_max = c->prof_n == 0 ? ms : std::max(c->prof_max, (double)ms);
        ++c->prof_n;
        c->prof_pool.push_back(e);
    }
    c->prof_pending.clear();
}

static void sn_need_device(const moc_sn_ctx *c) {
    if (c->host_only) throw Error(MOC_ESTATE, "host-only context (negative device ordinal): no device state");
}

static int sn_solve_impl(moc_sn_ctx *c, double tol, int max_iter, int check_every, moc_result *out) {
    if (!out) throw Error(MOC_EINVAL, "sn solve: null result");
    sn_need_device(c);
    SN_HIP(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    DevSN &d = c->d;
    hipStream_t s = c->stream;
    const bool eigen = c->fissile && !c->fixed_source;
    const int64_t nphi = (int64_t)d.T * d.G * 3, nb = d.nbnd * d.G * 3;
    c->cur_phi = 0;
    launch_sn_cold(d.phi[0], nphi, s);
    launch_sn_fill(d.bnd[0], nb, d.precision, s);
    launch_sn_fill(d.bnd[1], nb, d.precision, s);
    launch_sn_fill_f64(d.scal, kSnCount, 0.0, s);
    launch_sn_fill_f64(d.scal + kSnK, 1, 1.0, s);
    if (eigen) {
        launch_sn_fission_partials(d, d.phi[0], s);
        launch_sn_eigen_update(d, 0, s);
        launch_sn_scale_f64(d.phi[0], nphi, d.scal + kSnF, s);
    }
    int it = 0, sweeps = 0;
    bool conv = false;
    double res = 1.0, dk = 1.0, k = 1.0;
    for (it = 1; it <= max_iter; ++it) {
        double *phi_old = d.phi[c->cur_phi], *phi_new = d.phi[1 - c->cur_phi];
        launch_sn_source(d, phi_old, s);
        sn_sweep_impl(c, s);
        ++sweeps;
        launch_sn_finalize(d, phi_new, nullptr, d.partials, s);
        launch_sn_eigen_update(d, eigen ? 1 : 2, s);
        launch_sn_norm_residual(d, phi_new, phi_old, s);
        if (eigen) launch_sn_scale(d.bnd[c->cur_bnd], nb, d.precision, d.scal + kSnF, s);
        c->cur_phi = 1 - c->cur_phi;
        if (it % check_every == 0 || it == max_iter) {
            SN_HIP(hipMemcpyAsync(c->host_scal, d.scal, kSnCount * sizeof(double), hipMemcpyDeviceToHost, s));
            SN_HIP(hipStreamSynchronize(s));
            k = c->host_scal[kSnK];
            res = c->host_scal[kSnRes];
            dk = c->host_scal[kSnDk];
            if (!std::isfinite(res) || !std::isfinite(k)) throw Error(MOC_EHIP, "sn solve: non-finite iterate");
            if (res < tol && dk < tol) {
                conv = true;
                break;
            }
        }
    }
    out->k = eigen ? k : 1.0;
    out->iterations = conv ? it : max_iter;
    out->residual = res;
    out->dk = dk;
    out->flags = c->fixed_source ? MOC_FLAG_FIXED_SOURCE : 0;
    out->sweeps = sweeps;
    out->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return conv ? MOC_OK : MOC_ENOCONV;
}

extern "C" {

int moc_sn_create(const moc_mesh *mesh, const moc_tracks *angles, const moc_xs *xs, const moc_options *opts,
                  moc_sn_ctx **out) {
    if (!out) {
        g_sn_create_error = "sn create: null output pointer";
        return MOC_EINVAL;
    }
    *out = nullptr;
    moc_sn_ctx *c = new (std::nothrow) moc_sn_ctx();
    if (!c) {
        g_sn_create_error = "host allocation failed";
        return MOC_ENOMEM;
    }
    const int rc = sn_guarded(c, [&] { sn_create_impl(mesh, angles, xs, opts, c); });
    if (rc != MOC_OK) {
        g_sn_create_error = c->err;
        delete c;
        return rc;
    }
    g_sn_create_error.clear();
    *out = c;
    return MOC_OK;
}

void moc_sn_destroy(moc_sn_ctx *c) { delete c; }

int moc_sn_sweep(moc_sn_ctx *c, const double *source_dev, double *phi_out_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        if (!source_dev || !phi_out_dev) throw Error(MOC_EINVAL, "sn sweep: null pointer");
        sn_need_device(c);
        SN_HIP(hipSetDevice(c->device));
        hipStream_t s = stream ? (hipStream_t)stream : c->stream;
        launch_sn_prep_user(c->d, source_dev, s);
        sn_sweep_impl(c, s);
        launch_sn_finalize(c->d, nullptr, phi_out_dev, nullptr, s);
    });
}

int moc_sn_solve(moc_sn_ctx *c, double tol, moc_result *out) {
    if (!c) return MOC_EINVAL;
    int status = MOC_OK;
    const int rc = sn_guarded(c, [&] {
        if (!(tol > 0)) throw Error(MOC_EINVAL, "sn solve: tol must be positive");
        status = sn_solve_impl(c, tol, c->max_iter, c->check_every, out);
    });
    if (rc != MOC_OK) return rc;
    if (status != MOC_OK) c->err = "sn solve: not converged within max_iter";
    return status;
}

int moc_sn_run_iterations(moc_sn_ctx *c, int32_t n, moc_result *out) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        if (n <= 0) throw Error(MOC_EINVAL, "sn run_iterations: n must be positive");
        sn_solve_impl(c, 0.0, n, n, out);
    });
}

int moc_sn_get_flux(moc_sn_ctx *c, double *phi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        if (!phi_dev) throw Error(MOC_EINVAL, "sn get_flux: null pointer");
        sn_need_device(c);
        SN_HIP(hipSetDevice(c->device));
        hipStream_t s = stream ? (hipStream_t)stream : c->stream;
        SN_HIP(hipMemcpyAsync(phi_dev, c->d.phi[c->cur_phi], (size_t)c->d.T * c->d.G * 3 * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    });
}

int moc_sn_set_external_source(moc_sn_ctx *c, const double *q_dev) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        sn_need_device(c);
        SN_HIP(hipSetDevice(c->device));
        DevSN &d = c->d;
        if (!q_dev) {
            c->fixed_source = false;
            return;
        }
        if (!d.qext) d.qext = c->dalloc<double>((size_t)d.T * d.G * 3);
        SN_HIP(hipMemcpyAsync(d.qext, q_dev, (size_t)d.T * d.G * 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        SN_HIP(hipStreamSynchronize(c->stream));
        c->fixed_source = true;
    });
}

int moc_sn_get_info(const moc_sn_ctx *c, moc_sn_info *info) {
    if (!c || !info) return MOC_EINVAL;
    info->n_elements = c->d.T;
    info->n_directions = c->d.nd;
    info->n_groups = c->d.G;
    info->n_levels = c->d.nsteps;
    info->n_tasks = c->d.ntask;
    info->n_slots = c->d.nslot;
    info->n_boundary_faces = c->d.nd > 0 ? c->d.nbnd / c->d.nd : 0;
    info->device_bytes = c->device_bytes;
    info->setup_ms = c->setup_ms;
    info->tasks_per_thread = c->d.tgroup;
    info->n_tiles = c->tiled ? c->tl.n_tiles : 0;
    info->n_tile_levels = c->tiled ? c->tl.n_levels : 0;
    info->max_inner_levels = c->tiled ? c->tl.max_inner : 0;
    info->tile_lds_bytes = c->tiled ? (int32_t)c->tl.lds_bytes : 0;
    info->n_tile_slots = c->tiled ? c->tl.nslot : 0;
    return MOC_OK;
}

int moc_sn_set_tiles(moc_sn_ctx *c, int32_t n_tiles, const int32_t *element_tile) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] { sn_set_tiles_impl(c, n_tiles, element_tile); });
}

int moc_sn_set_profiling(moc_sn_ctx *c, int32_t enable) {
    if (!c) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        sn_drain_profile(c);
        c->profiling = enable != 0;
        c->prof_n = 0;
        c->prof_ms = c->prof_min = c->prof_max = 0;
    });
}

int moc_sn_get_profile(moc_sn_ctx *c, moc_profile *out) {
    if (!c || !out) return MOC_EINVAL;
    return sn_guarded(c, [&] {
        sn_drain_profile(c);
        std::memset(out, 0, sizeof *out);
        out->sweeps = c->prof_n;
        out->sweep_ms = c->prof_ms;
        out->sweep_ms_min = c->prof_min;
        out->sweep_ms_max = c->prof_max;
    });
}

const char *moc_sn_last_error(const moc_sn_ctx *c) { return c ? c->err.c_str() : g_sn_create_error.c_str(); }

}  // extern "C"
