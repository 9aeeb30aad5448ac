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

struct moc_sn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevSN d;
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
    // runs of tgroup tasks and, per element, its runs (the scalar flux is gathered from them)
    d.nrun = ntask / d.tgroup;
    {
        std::vector<int> off((size_t)T + 1, 0), runs((size_t)d.nrun);
        for (int64_t r = 0; r < d.nrun; ++r) ++off[(size_t)task_e[(size_t)(r * d.tgroup)] + 1];
        for (int e = 0; e < T; ++e) off[(size_t)e + 1] += off[(size_t)e];
        std::vector<int> fill(off.begin(), off.end() - 1);
        for (int64_t r = 0; r < d.nrun; ++r) runs[(size_t)fill[(size_t)task_e[(size_t)(r * d.tgroup)]]++] = (int)r;
        d.elem_off = c->upload(off);
        d.elem_runs = c->upload(runs);
    }
    d.run_acc = f64 ? (void *)c->dalloc<double>((size_t)d.nrun * G * 3) : (void *)c->dalloc<float>((size_t)d.nrun * G * 3);
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
// (every direction's elements of that level, all groups), then the gather of the scalar
// flux; reflective inflow reads boundary buffer `parity`, outflow writes the other.
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
    for (int st = 0; st < d.nsteps; ++st) {
        a.k0 = d.step_off[st];
        a.k1 = d.step_off[st + 1];
        launch_sn_step(a, d.precision, s);
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
    return MOC_OK;
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
