// C ABI of libmoc's DGMOC solver (declared in include/dgmoc.h): context creation on top of
// the planar context (mesh, tracks, packing), the per-plane sweep sequence of
// Alg. DGMOC_sweep, and the power / source iteration. No exception crosses the ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "dg_kernels.h"
#include "dgmoc.h"
#include "moc_ctx.h"

using namespace moc;

struct moc_dg_ctx {
    moc_ctx base;   // planar geometry, tracks, packing and shared device arrays (XS, V, scalars)
    DevDG g;
    int cur_psi = 0, cur_phi = 0;
    bool fixed_source = false;
    double setup_ms = 0;
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_pool;
    int64_t prof_n = 0;
    double prof_ms = 0, prof_min = 0, prof_max = 0;
    ~moc_dg_ctx() {
        if (base.stream) hipStreamSynchronize(base.stream);
        for (auto *v : {&prof_pending, &prof_pool})
            for (auto &e : *v) {
                hipEventDestroy(e.first);
                hipEventDestroy(e.second);
            }
    }
};

static thread_local std::string g_dg_create_error;

static int dg_guarded(moc_dg_ctx *c, const std::function<void()> &f) { return guarded_call(c ? &c->base : nullptr, f); }

namespace {

// Per-angle track area Va[a][r] = sum over the angle's segments in r of delta_a l, by
// tracing every track again (threads own whole angles, so rows are written by one thread).
struct VaSink : SegmentSink {
    double *row = nullptr;
    const int *internal_of_user = nullptr;
    double delta = 0;
    void emit(int region, double length) override { row[internal_of_user[region]] += delta * length; }
};

}  // namespace

static void dg_create_impl(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs, const moc_axial *ax,
                           const moc_options *opt, moc_dg_ctx *c) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!mesh || !tracks || !xs || !ax) throw Error(MOC_EINVAL, "dg create: null argument");
    moc_options o{};
    if (opt) o = *opt;
    if (o.device < 0) throw Error(MOC_EINVAL, "dg create: a device ordinal >= 0 is required");
    // defaults measured on the 17 x 17 x 16-plane workload: two groups per wavefront and
    // the largest tally windows (fewer flushes and padding steps; more wavefronts in flight)
    if (o.tally_slots == 0) o.tally_slots = 256;
    if (o.group_batch == 0) o.group_batch = 2;
    if (o.group_batch != 1 && o.group_batch != 2 && o.group_batch != 4)
        throw Error(MOC_EINVAL, "dg options: group_batch must be 0, 1, 2 or 4");
    const int Nz = ax->n_planes;
    if (Nz < 1 || !ax->dz) throw Error(MOC_EINVAL, "axial: n_planes must be >= 1 and dz non-null");
    for (int z = 0; z < Nz; ++z)
        if (!(ax->dz[z] > 0) || !std::isfinite(ax->dz[z])) throw Error(MOC_EINVAL, "axial: plane heights must be positive");
    if ((ax->bc_bottom != MOC_BC_VACUUM && ax->bc_bottom != MOC_BC_REFLECTIVE) ||
        (ax->bc_top != MOC_BC_VACUUM && ax->bc_top != MOC_BC_REFLECTIVE))
        throw Error(MOC_EINVAL, "axial: bad boundary condition");
    if (ax->angle_block < 0) throw Error(MOC_EINVAL, "axial: angle_block must be >= 0");
    if (ax->plane_material)
        for (int64_t i = 0; i < (int64_t)Nz * mesh->n_regions; ++i)
            if (ax->plane_material[i] < 0 || ax->plane_material[i] >= xs->n_materials)
                throw Error(MOC_EINVAL, "axial: plane material out of range");

    create_context(mesh, tracks, xs, &o, &c->base);
    moc_ctx &b = c->base;
    DevProblem &d = b.d;
    DevDG &g = c->g;
    const int R = d.R, G = d.G, P = d.P, NA = d.NA;
    g.Nz = Nz;
    g.dz.assign(ax->dz, ax->dz + Nz);
    g.bc_bot = ax->bc_bottom;
    g.bc_top = ax->bc_top;
    g.gb = d.gb;
    g.n_gb = d.n_gb;
    g.Gp = d.Gp;
    for (int p = 0; p < P; ++p) g.mu[p] = b.quad.mu[p];

    // angle blocks: batches are in canonical track order, which is by angle
    const std::vector<int> &ba = b.host_batch_angle;
    for (size_t i = 1; i < ba.size(); ++i)
        if (ba[i] < ba[i - 1]) throw Error(MOC_EINVAL, "dg create: batches are not ordered by angle");
    g.nab = ax->angle_block > 0 ? std::min(ax->angle_block, NA) : NA;
    g.n_blocks = (NA + g.nab - 1) / g.nab;
    g.blk_angle0.assign(g.n_blocks + 1, NA);
    g.blk_batch0.assign(g.n_blocks + 1, d.nb);
    for (int k = 0; k < g.n_blocks; ++k) {
        g.blk_angle0[k] = k * g.nab;
        g.blk_batch0[k] = int(std::lower_bound(ba.begin(), ba.end(), k * g.nab) - ba.begin());
    }

    // per (plane, region): material, V h, Sigma_t (padded groups: 1)
    const bool f64 = d.precision == MOC_PREC_F64;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);
    std::vector<int> mat3((size_t)Nz * R);
    std::vector<double> hV((size_t)Nz * R), V_int(R);
    for (int r = 0; r < R; ++r) V_int[r] = b.V_user[b.user_of_internal[r]];
    for (int z = 0; z < Nz; ++z)
        for (int r = 0; r < R; ++r) {
            const int u = b.user_of_internal[r];
            mat3[(size_t)z * R + r] = ax->plane_material ? ax->plane_material[(size_t)z * R + u] : mesh->region_material[u];
            hV[(size_t)z * R + r] = V_int[r] * g.dz[z];
        }
    std::vector<double> st3((size_t)Nz * R * g.Gp, 1.0);
    for (size_t c3 = 0; c3 < mat3.size(); ++c3)
        for (int gg = 0; gg < G; ++gg) st3[c3 * g.Gp + gg] = b.sigt_m_host[(size_t)mat3[c3] * G + gg];
    g.mat3 = b.upload(mat3);
    g.hV = b.upload(hV);

    // per-angle track areas
    std::vector<double> Va((size_t)NA * R, 0.0);
    std::vector<int> angle_first(NA + 1, b.tracks.T);
    for (int t = b.tracks.T - 1; t >= 0; --t) angle_first[b.tracks.angle[t]] = t;
    for (int a = NA - 1; a >= 0; --a)
        if (angle_first[a] > angle_first[a + 1]) angle_first[a] = angle_first[a + 1];
    parallel_for(NA, b.n_threads, 1, [&](int64_t a0, int64_t a1, int) {
        VaSink sink;
        sink.internal_of_user = b.internal_of_user.data();
        for (int64_t a = a0; a < a1; ++a) {
            sink.row = Va.data() + (size_t)a * R;
            sink.delta = b.quad.delta[a];
            for (int t = angle_first[a]; t < angle_first[a + 1]; ++t) trace_track(b.mesh, b.quad, b.tracks, t, sink);
        }
    });
    std::vector<double> inv_va(Va.size()), wdir((size_t)NA * P), dlt(NA);
    for (size_t i = 0; i < Va.size(); ++i) inv_va[i] = Va[i] > 0 ? 1.0 / Va[i] : 0.0;
    for (int a = 0; a < NA; ++a) {
        dlt[a] = b.quad.delta[a];
        for (int p = 0; p < P; ++p)
            wdir[(size_t)a * P + p] = 3.14159265358979323846 * b.quad.wa[a] * b.quad.wp[p] * b.quad.delta[a];
    }
    auto up_real = [&](const std::vector<double> &v) -> void * {
        if (f64) return b.upload(v);
        return b.upload(std::vector<float>(v.begin(), v.end()));
    };
    g.sigt3 = up_real(st3);
    g.inv_va = up_real(inv_va);
    g.wdir = up_real(wdir);
    g.dlt = up_real(dlt);

    // work arrays
    const int64_t ncell = (int64_t)Nz * R;
    g.q3 = b.dalloc<char>((size_t)ncell * g.Gp * 2 * rs);
    g.face_count = (int64_t)2 * g.nab * P * R * g.Gp;
    g.face = b.dalloc<char>((size_t)g.face_count * rs);
    g.drv = b.dalloc<char>((size_t)2 * g.nab * R * g.n_gb * P * g.gb * 2 * rs);
    if (g.bc_bot == MOC_BC_REFLECTIVE) {
        g.bot_count = (int64_t)2 * NA * P * R * g.Gp;
        g.bot = b.dalloc<char>((size_t)g.bot_count * rs);
    }
    g.tally = b.dalloc<double>((size_t)ncell * g.Gp * 2);
    g.phi[0] = b.dalloc<double>((size_t)ncell * G * 2);
    g.phi[1] = b.dalloc<double>((size_t)ncell * G * 2);
    g.psi_count = (int64_t)2 * Nz * 2 * P * 2 * g.Gp * d.nslots;
    g.psi[0] = b.dalloc<char>((size_t)g.psi_count * rs);
    g.psi[1] = b.dalloc<char>((size_t)g.psi_count * rs);
    hipStream_t s = b.stream;
    launch_fill_real(g.q3, ncell * g.Gp * 2, d.precision, s);
    launch_fill_real(g.face, g.face_count, d.precision, s);
    if (g.bot) launch_fill_real(g.bot, g.bot_count, d.precision, s);
    launch_fill_real(g.psi[0], g.psi_count, d.precision, s);
    launch_fill_real(g.psi[1], g.psi_count, d.precision, s);
    launch_dg_cold_flux(g, g.phi[0], ncell * G * 2, s);
    HIP_OK(hipStreamSynchronize(s));
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static std::pair<hipEvent_t, hipEvent_t> dg_prof_events(moc_dg_ctx *c) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->prof_pool.empty()) {
        HIP_OK(hipEventCreate(&ev.first));
        HIP_OK(hipEventCreate(&ev.second));
    } else {
        ev = c->prof_pool.back();
        c->prof_pool.pop_back();
    }
    return ev;
}

// One transport sweep with the emission in g.q3 (Alg. DGMOC_sweep): per angle block,
// per ward, per plane in sweep order: driven flux (face flux entering the plane), ray
// tracing with tallies of both moments and of the face flux leaving the plane; after the
// downward ward, the flux leaving through the bottom is kept for a reflective bottom.
static void dg_sweep_impl(moc_dg_ctx *c, hipStream_t s) {
    moc_ctx &b = c->base;
    DevProblem &d = b.d;
    DevDG &g = c->g;
    const int R = d.R, P = d.P;
    const size_t rs = d.precision == MOC_PREC_F64 ? sizeof(double) : sizeof(float);
    const int64_t plane_psi = (int64_t)2 * P * 2 * g.Gp * d.nslots;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->profiling) {
        ev = dg_prof_events(c);
        HIP_OK(hipEventRecord(ev.first, s));
    }
    launch_fill_f64(g.tally, (int64_t)g.Nz * R * g.Gp * 2, 0.0, s);
    DgDrivenArgs da{};
    da.face = g.face;
    da.bot = g.bot;
    da.inv_va = g.inv_va;
    da.drv = g.drv;
    da.R = R;
    da.P = P;
    da.Gp = g.Gp;
    da.gb = g.gb;
    da.n_gb = g.n_gb;
    DgSweepArgs sa{};
    sa.segs = d.segs;
    sa.batch_win = d.batch_win;
    sa.win_entry_off = d.win_entry_off;
    sa.win_tab_off = d.win_tab_off;
    sa.win_nsteps = d.win_nsteps;
    sa.win_nslots = d.win_nslots;
    sa.win_tab = d.win_tab;
    sa.cap = d.max_slots;
    sa.batch_angle = d.batch_angle;
    sa.drv = g.drv;
    sa.link = d.link;
    sa.fed = d.fed;
    sa.wdir = g.wdir;
    sa.dlt = g.dlt;
    sa.inv_sin = d.inv_sin;
    sa.face = g.face;
    sa.nslots = d.nslots;
    sa.Gp = g.Gp;
    sa.R = R;
    sa.n_gb = g.n_gb;
    char *psi_in = static_cast<char *>(g.psi[c->cur_psi]), *psi_out = static_cast<char *>(g.psi[1 - c->cur_psi]);
    for (int k = 0; k < g.n_blocks; ++k) {
        const int a0 = g.blk_angle0[k], a1 = g.blk_angle0[k + 1];
        const int b0 = g.blk_batch0[k], nbk = g.blk_batch0[k + 1] - b0;
        da.a0 = a0;
        da.nab = a1 - a0;
        sa.a0 = a0;
        sa.b0 = b0;
        for (int w = 0; w < 2; ++w) {
            const double sgn = w == 0 ? 1.0 : -1.0;
            da.sgn = sa.sgn = sgn;
            for (int n = 0; n < g.Nz; ++n) {
                const int z = w == 0 ? n : g.Nz - 1 - n;
                for (int p = 0; p < P; ++p) da.kap[p] = sa.kap[p] = g.mu[p] / g.dz[z];
                if (n > 0)
                    da.mode = 1;
                else if (w == 0)
                    da.mode = g.bc_bot == MOC_BC_REFLECTIVE ? 2 : 0;
                else
                    da.mode = g.bc_top == MOC_BC_REFLECTIVE ? 1 : 0;
                da.sigt = sa.sigt = static_cast<char *>(g.sigt3) + (size_t)z * R * g.Gp * rs;
                da.q = static_cast<char *>(g.q3) + (size_t)z * R * g.Gp * 2 * rs;
                launch_dg_driven(da, d.precision, s);
                const int64_t off = ((int64_t)w * g.Nz + z) * plane_psi * (int64_t)rs;
                sa.psi_in = psi_in + off;
                sa.psi_out = psi_out + off;
                sa.tally = g.tally + (size_t)z * R * g.Gp * 2;
                launch_dg_sweep(sa, d.precision, nbk, P, g.gb, s);
            }
            if (w == 1 && g.bc_bot == MOC_BC_REFLECTIVE) launch_dg_store_bottom(da, d.precision, s);
        }
    }
    c->cur_psi = 1 - c->cur_psi;
    if (c->profiling) {
        HIP_OK(hipEventRecord(ev.second, s));
        c->prof_pending.push_back(ev);
    }
}

static void dg_drain_profile(moc_dg_ctx *c) {
    for (auto &e : c->prof_pending) {
        HIP_OK(hipEventSynchronize(e.second));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_ms += ms;
        c->prof_min = c->prof_n == 0 ? ms : std::min(c->prof_min, (double)ms);
        c->prof_max = c->prof_n == 0 ? ms : std::max(c->prof_max, (double)ms);
        ++c->prof_n;
        c->prof_pool.push_back(e);
    }
    c->prof_pending.clear();
}

static int dg_solve_impl(moc_dg_ctx *c, double tol, int max_iter, int check_every, moc_result *out) {
    if (!out) throw Error(MOC_EINVAL, "dg solve: null result");
    moc_ctx &b = c->base;
    HIP_OK(hipSetDevice(b.device));
    const auto t0 = std::chrono::steady_clock::now();
    DevProblem &d = b.d;
    DevDG &g = c->g;
    hipStream_t s = b.stream;
    const bool eigen = b.fissile && !c->fixed_source;
    const int64_t nphi = (int64_t)g.Nz * d.R * d.G * 2;
    c->cur_phi = 0;
    launch_dg_cold_flux(g, g.phi[0], nphi, s);
    launch_fill_real(g.psi[0], g.psi_count, d.precision, s);
    launch_fill_real(g.psi[1], g.psi_count, d.precision, s);
    if (g.bot) launch_fill_real(g.bot, g.bot_count, d.precision, s);
    launch_fill_f64(d.scal, kScalCount, 0.0, s);
    launch_fill_f64(d.scal + kScalK, 1, 1.0, s);
    if (eigen) {
        launch_dg_fission_partials(d, g, g.phi[0], d.partials, s);
        launch_eigen_update(d, d.partials, 0, s);
        launch_scale_f64(g.phi[0], nphi, d.scal + kScalF, s);
    }
    int it = 0, sweeps = 0;
    bool conv = false;
    double res = 1.0, dk = 1.0, k = 1.0;
    for (it = 1; it <= max_iter; ++it) {
        double *phi_old = g.phi[c->cur_phi], *phi_new = g.phi[1 - c->cur_phi];
        launch_dg_source(d, g, phi_old, s);
        dg_sweep_impl(c, s);
        ++sweeps;
        launch_dg_finalize(d, g, phi_new, nullptr, d.partials, s);
        launch_eigen_update(d, d.partials, eigen ? 1 : 2, s);
        launch_dg_norm_residual(d, g, phi_new, phi_old, d.partials, s);
        if (eigen) {
            launch_scale_real(g.psi[c->cur_psi], g.psi_count, d.precision, d.scal + kScalF, s);
            if (g.bot) launch_scale_real(g.bot, g.bot_count, d.precision, d.scal + kScalF, s);
        }
        c->cur_phi = 1 - c->cur_phi;
        if (it % check_every == 0 || it == max_iter) {
            HIP_OK(hipMemcpyAsync(b.host_scal, d.scal, kScalCount * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            k = b.host_scal[kScalK];
            res = b.host_scal[kScalRes];
            dk = b.host_scal[kScalDk];
            if (!std::isfinite(res) || !std::isfinite(k)) throw Error(MOC_EHIP, "dg solve: non-finite iterate");
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

int moc_dg_create(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs, const moc_axial *axial,
                  const moc_options *opts, moc_dg_ctx **out) {
    if (!out) {
        g_dg_create_error = "dg create: null output pointer";
        return MOC_EINVAL;
    }
    *out = nullptr;
    moc_dg_ctx *c = new (std::nothrow) moc_dg_ctx();
    if (!c) {
        g_dg_create_error = "host allocation failed";
        return MOC_ENOMEM;
    }
    const int rc = dg_guarded(c, [&] { dg_create_impl(mesh, tracks, xs, axial, opts, c); });
    if (rc != MOC_OK) {
        g_dg_create_error = c->base.err;
        delete c;
        return rc;
    }
    g_dg_create_error.clear();
    *out = c;
    return MOC_OK;
}

void moc_dg_destroy(moc_dg_ctx *c) { delete c; }

int moc_dg_sweep(moc_dg_ctx *c, const double *source_dev, double *phi_out_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        if (!source_dev || !phi_out_dev) throw Error(MOC_EINVAL, "dg sweep: null pointer");
        HIP_OK(hipSetDevice(c->base.device));
        hipStream_t s = stream ? (hipStream_t)stream : c->base.stream;
        launch_dg_prep_user(c->base.d, c->g, source_dev, s);
        dg_sweep_impl(c, s);
        launch_dg_finalize(c->base.d, c->g, nullptr, phi_out_dev, nullptr, s);
    });
}

int moc_dg_solve(moc_dg_ctx *c, double tol, moc_result *out) {
    if (!c) return MOC_EINVAL;
    int status = MOC_OK;
    const int rc = dg_guarded(c, [&] {
        if (!(tol > 0)) throw Error(MOC_EINVAL, "dg solve: tol must be positive");
        status = dg_solve_impl(c, tol, c->base.max_iter, c->base.check_every, out);
    });
    if (rc != MOC_OK) return rc;
    if (status != MOC_OK) c->base.err = "dg solve: not converged within max_iter";
    return status;
}

int moc_dg_run_iterations(moc_dg_ctx *c, int32_t n, moc_result *out) {
    if (!c) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        if (n <= 0) throw Error(MOC_EINVAL, "dg run_iterations: n must be positive");
        dg_solve_impl(c, 0.0, n, n, out);
    });
}

int moc_dg_get_flux(moc_dg_ctx *c, double *phi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        if (!phi_dev) throw Error(MOC_EINVAL, "dg get_flux: null pointer");
        HIP_OK(hipSetDevice(c->base.device));
        hipStream_t s = stream ? (hipStream_t)stream : c->base.stream;
        launch_dg_permute(c->base.d, c->g, c->g.phi[c->cur_phi], phi_dev, 1, s);
    });
}

int moc_dg_set_external_source(moc_dg_ctx *c, const double *q_dev) {
    if (!c) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        moc_ctx &b = c->base;
        HIP_OK(hipSetDevice(b.device));
        if (!q_dev) {
            b.dfree(c->g.qext);
            c->g.qext = nullptr;
            c->fixed_source = false;
            return;
        }
        if (!c->g.qext) c->g.qext = b.dalloc<double>((size_t)c->g.Nz * b.d.R * b.d.G * 2);
        launch_dg_permute(b.d, c->g, q_dev, c->g.qext, 0, b.stream);
        HIP_OK(hipStreamSynchronize(b.stream));
        c->fixed_source = true;
    });
}

int moc_dg_get_info(const moc_dg_ctx *c, moc_dg_info *info) {
    if (!c || !info) return MOC_EINVAL;
    const DevProblem &d = c->base.d;
    info->n_planes = c->g.Nz;
    info->n_blocks = c->g.n_blocks;
    info->angles_per_block = c->g.nab;
    info->group_batch = c->g.gb;
    info->n_updates = 2LL * 2LL * d.P * d.G * c->base.S * c->g.Nz;
    info->device_bytes = c->base.device_bytes;
    info->setup_ms = c->setup_ms;
    return MOC_OK;
}

int moc_dg_set_profiling(moc_dg_ctx *c, int32_t enable) {
    if (!c) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        dg_drain_profile(c);
        c->profiling = enable != 0;
        c->prof_n = 0;
        c->prof_ms = c->prof_min = c->prof_max = 0;
    });
}

int moc_dg_get_profile(moc_dg_ctx *c, moc_profile *out) {
    if (!c || !out) return MOC_EINVAL;
    return dg_guarded(c, [&] {
        dg_drain_profile(c);
        std::memset(out, 0, sizeof *out);
        out->sweeps = c->prof_n;
        out->sweep_ms = c->prof_ms;
        out->sweep_ms_min = c->prof_min;
        out->sweep_ms_max = c->prof_max;
    });
}

const char *moc_dg_last_error(const moc_dg_ctx *c) { return c ? c->base.err.c_str() : g_dg_create_error.c_str(); }

}  // extern "C"
