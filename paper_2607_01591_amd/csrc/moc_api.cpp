// C ABI of libmoc (declared in include/moc.h): context creation (host setup + device
// packing), sweep, power/source iteration, state access. No exception crosses the ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>

#include "moc_ctx.h"

using namespace moc;

static thread_local std::string g_create_error;

// transport sweeps with a frozen source that precede a warm start without boundary fluxes
static constexpr int kWarmBoundarySweeps = 2;
// iterations of a warm start whose residual is compared with the cold start's first one
static constexpr int kGuessWatch = 10;

// default lane stagger of the tally windows (moc_options.lane_stagger = 0)
static constexpr int kDefaultLaneStagger = 2;

template <typename F> static int guarded(moc_ctx *ctx, F &&f) {
    try {
        f();
        if (ctx) ctx->err.clear();
        return MOC_OK;
    } catch (const Error &e) {
        if (ctx) ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        return MOC_ENOMEM;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = e.what();
        return MOC_EINVAL;
    } catch (...) {
        if (ctx) ctx->err = "unknown error";
        return MOC_EINVAL;
    }
}

// Workgroups are handed to the chip's 8 XCDs round robin by their linear index, and each
// XCD has its own L2. Order 1 gives XCD x (the workgroup columns x, x + 8, ...) one
// contiguous range of batches, i.e. neighbouring tracks whose segments gather the same
// regions' cross sections; order 0 (default) keeps batch = column, which measured as fast
// or faster on the 51 x 51 lattice (the gathered rows are served from the shared
// infinity cache either way).
static constexpr int kXcds = 8;
static std::vector<int> make_batch_order(int nb, int order) {
    std::vector<int> b(nb);
    if (order == 0) {
        for (int i = 0; i < nb; ++i) b[i] = i;
        return b;
    }
    int start = 0;
    for (int x = 0; x < kXcds; ++x) {
        const int count = nb > x ? (nb - x + kXcds - 1) / kXcds : 0;   // columns i = x mod 8
        for (int k = 0; k < count; ++k) b[x + kXcds * k] = start + k;
        start += count;
    }
    return b;
}

// One batch when an instance holds all groups; otherwise batches of 8 (float4 row loads,
// 184 VGPRs at 3 polar angles) unless 7 divides G exactly. On the 33-group hexagon a
// sweep takes 9.3 ms in batches of 8 (7 padding groups), 11.0 ms in batches of 11 (234
// VGPRs), 12.6 ms of 7 and 14.3 ms of 4.
static int choose_group_batch(int G) {
    if (G == 1 || G == 2 || G == 4 || G == 7 || G == 8 || G == 11) return G;
    if (G == 3) return 4;
    if (G <= 8) return 8;
    if (G % 8 == 0) return 8;
    if (G % 7 == 0) return 7;
    return 8;
}

namespace {

struct DumpSink : SegmentSink {
    std::vector<int> reg;
    std::vector<double> len;
    void emit(int r, double l) override {
        reg.push_back(r);
        len.push_back(l);
    }
};

}  // namespace

// Trace, cut into tally windows and pack every batch (two deterministic passes), then load
// the segment stream and the window tables on the device, replacing any previous ones.
// With `coarse`, the stream carries coarse-surface crossing entries.
static void pack_and_upload(moc_ctx *c, const CoarseSurfaces *coarse, PackOutput &pk) {
    DevProblem &d = c->d;
    PackInput pin = c->pin;
    pin.coarse = coarse;
    for (void *p : {d.segs, (void *)d.batch_win, (void *)d.win_entry_off, (void *)d.win_nsteps, (void *)d.win_tab_off,
                    (void *)d.win_nslots, (void *)d.win_tab, (void *)d.entry_region})
        c->dfree(p);
    if (d.precision == MOC_PREC_F64) {
        std::vector<SegD> segs;
        pack_segments_f64(pin, pk, segs);
        d.segs = c->upload(segs);
        if (c->host_only) c->host_segs_f64.swap(segs);
    } else {
        std::vector<SegF> segs;
        pack_segments_f32(pin, pk, segs);
        d.segs = c->upload(segs);
        if (c->host_only) c->host_segs_f32.swap(segs);
    }
    c->S = pk.S;
    c->crossings = pk.crossings;
    c->padded_steps = pk.entries;
    c->window_len = pin.window_len;
    c->n_windows = (int64_t)pk.win_nsteps.size();
    c->n_slots_total = (int64_t)pk.tab.size();
    int max_slots = 1;
    for (int v : pk.win_nslots) max_slots = std::max(max_slots, v);
    d.max_slots = max_slots;
    d.batch_win = c->upload(pk.batch_win);
    d.win_entry_off = c->upload(pk.win_entry_off);
    d.win_nsteps = c->upload(pk.win_nsteps);
    d.win_tab_off = c->upload(pk.win_tab_off);
    d.win_nslots = c->upload(pk.win_nslots);
    d.win_tab = c->upload(pk.tab);
    d.entry_region = c->upload(pk.entry_region);
    if (c->host_only) c->host_pack = pk;
}

void moc::create_context(const moc_mesh *mesh_in, const moc_tracks *tr_in, const moc_xs *xs, const moc_options *opt,
                        moc_ctx *c) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!mesh_in || !tr_in || !xs) throw Error(MOC_EINVAL, "create: null argument");
    moc_options o{};
    o.precision = MOC_PREC_F32;
    o.exp_mode = MOC_EXP_POLY;
    if (opt) o = *opt;
    if (o.tally_slots != 0 && (o.tally_slots < kBatch || o.tally_slots > kMaxSlots))
        throw Error(MOC_EINVAL, "options: tally_slots must be 0 or in 64..256");
    if (o.precision != MOC_PREC_F32 && o.precision != MOC_PREC_F64) throw Error(MOC_EINVAL, "options: bad precision");
    if (o.exp_mode < MOC_EXP_POLY || o.exp_mode > MOC_EXP_DIFF) throw Error(MOC_EINVAL, "options: bad exp_mode");
    c->max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    c->check_every = o.check_every > 0 ? o.check_every : 1;
    c->n_threads = o.n_threads > 0 ? o.n_threads : std::max(1u, std::thread::hardware_concurrency());
    c->device = o.device;
    c->host_only = o.device < 0;
    if (!c->host_only) {
        HIP_OK(hipSetDevice(c->device));
        HIP_OK(hipStreamCreate(&c->stream));
        HIP_OK(hipHostMalloc((void **)&c->host_scal, kScalCount * sizeof(double)));
    }

    // ---- cross sections
    const int M = xs->n_materials, G = xs->n_groups;
    if (M <= 0 || G <= 0 || !xs->sigma_t || !xs->sigma_s || !xs->nu_sigma_f || !xs->chi)
        throw Error(MOC_EINVAL, "xs: empty or null arrays");
    for (int i = 0; i < M * G; ++i)
        if (!(xs->sigma_t[i] > 0) || !std::isfinite(xs->sigma_t[i])) throw Error(MOC_EINVAL, "xs: Sigma_t must be positive and finite");
    for (int i = 0; i < M * G * G; ++i)
        if (!std::isfinite(xs->sigma_s[i])) throw Error(MOC_EINVAL, "xs: non-finite Sigma_s");
    for (int i = 0; i < M * G; ++i)
        if (!std::isfinite(xs->nu_sigma_f[i]) || !std::isfinite(xs->chi[i])) throw Error(MOC_EINVAL, "xs: non-finite nuSigma_f or chi");
    c->sigt_m_host.assign(xs->sigma_t, xs->sigma_t + M * G);
    c->nsf_m_host.assign(xs->nu_sigma_f, xs->nu_sigma_f + M * G);
    for (int i = 0; i < M * G; ++i) c->fissile |= xs->nu_sigma_f[i] > 0;

    // ---- geometry and tracks (host)
    build_mesh(*mesh_in, c->mesh);
    if (!mesh_in->region_material) throw Error(MOC_EINVAL, "mesh: null region_material");
    for (int r = 0; r < c->mesh.R; ++r)
        if (mesh_in->region_material[r] < 0 || mesh_in->region_material[r] >= M)
            throw Error(MOC_EINVAL, "mesh: material index out of range");
    build_quadrature(c->mesh, *tr_in, c->quad);
    lay_tracks(c->mesh, c->quad, c->tracks);
    link_tracks(c->mesh, c->quad, c->tracks);
    locality_order(c->mesh, c->internal_of_user, c->user_of_internal);

    DevProblem &d = c->d;
    const int R = c->mesh.R, T = c->tracks.T, P = c->quad.P;
    d.R = R;
    d.G = G;
    d.M = M;
    d.P = P;
    d.NA = c->quad.NA;
    d.T = T;
    d.precision = o.precision;
    d.exp_mode = o.exp_mode;
    if (o.group_batch != 0 && o.group_batch != 1 && o.group_batch != 2 && o.group_batch != 4 && o.group_batch != 7 &&
        o.group_batch != 8 && o.group_batch != 11)
        throw Error(MOC_EINVAL, "options: group_batch must be 0, 1, 2, 4, 7, 8 or 11");
    d.gb = o.group_batch > 0 ? o.group_batch : choose_group_batch(G);
    d.n_gb = (G + d.gb - 1) / d.gb;
    d.Gp = ((d.n_gb * d.gb + 3) / 4) * 4;
    const bool f64 = o.precision == MOC_PREC_F64;
    const size_t rs = f64 ? sizeof(double) : sizeof(float);

    // ---- batches: 64 consecutive tracks of one angle per batch
    std::vector<int> batch_angle, batch_of_track(T);
    c->slot_of_canon.assign(T, -1);
    for (int t = 0; t < T;) {
        const int a = c->tracks.angle[t];
        int e = t;
        while (e < T && c->tracks.angle[e] == a) ++e;
        for (int s = t; s < e; s += kBatch) {
            const int b = (int)batch_angle.size();
            batch_angle.push_back(a);
            for (int k = s; k < std::min(e, s + kBatch); ++k) {
                batch_of_track[k] = b;
                c->slot_of_canon[k] = b * kBatch + (k - s);
            }
        }
        t = e;
    }
    d.nb = (int)batch_angle.size();
    d.nslots = d.nb * kBatch;
    if (d.nb == 0) throw Error(MOC_EINVAL, "tracks: no track crosses the domain");
    std::vector<int> canon_of_slot(d.nslots, -1);
    for (int t = 0; t < T; ++t) canon_of_slot[c->slot_of_canon[t]] = t;

    // ---- trace, cut into tally windows, pack (two deterministic passes over batches)
    PackInput pin;
    pin.mesh = &c->mesh;
    pin.quad = &c->quad;
    pin.tracks = &c->tracks;
    pin.internal_of_user = c->internal_of_user.data();
    pin.n_threads = c->n_threads;
    pin.cap = o.tally_slots > 0 ? o.tally_slots : 256;
    if (o.window_steps < 0) throw Error(MOC_EINVAL, "options: window_steps must be >= 0");
    pin.window_steps = o.window_steps;
    if (o.lane_stagger < 0 || o.lane_stagger > kBatch) throw Error(MOC_EINVAL, "options: lane_stagger must be in 0..64");
    if (o.batch_order < 0 || o.batch_order > 1) throw Error(MOC_EINVAL, "options: batch_order must be 0 or 1");
    pin.stagger = o.lane_stagger > 0 ? o.lane_stagger : kDefaultLaneStagger;
    {
        double total_len = 0;
        for (int t = 0; t < T; ++t) total_len += c->tracks.len[t];
        pin.window_len = o.window_cm > 0 ? o.window_cm : 0.0;
        if (pin.window_len <= 0) {
            // about 32 segments per lane per window: estimate the mean segment length
            // from a sample of tracks
            struct Cnt : SegmentSink {
                int64_t n = 0;
                void emit(int, double) override { ++n; }
            } cnt;
            double len = 0;
            const int stride = std::max(1, T / 512);
            for (int t = 0; t < T; t += stride) {
                trace_track(c->mesh, c->quad, c->tracks, t, cnt);
                len += c->tracks.len[t];
            }
            pin.window_len = 32.0 * len / std::max<int64_t>(1, cnt.n);
        }
    }
    pin.batch_first.assign(d.nb + 1, T);
    for (int t = T - 1; t >= 0; --t) pin.batch_first[batch_of_track[t]] = t;
    c->pin = pin;
    d.cap = pin.cap;
    PackOutput pk;
    pack_and_upload(c, nullptr, pk);
    std::vector<double> &V_internal = pk.V;
    for (int r = 0; r < R; ++r)
        if (!(V_internal[r] > 0))
            throw Error(MOC_EINVAL, "tracking: region " + std::to_string(c->user_of_internal[r]) +
                                        " is crossed by no track (refine the track spacing)");
    c->V_user.assign(R, 0.0);
    for (int r = 0; r < R; ++r) c->V_user[c->user_of_internal[r]] = V_internal[r];
    d.batch_angle = c->upload(batch_angle);
    d.batch_of_block = c->upload(make_batch_order(d.nb, o.batch_order));
    c->host_batch_angle = batch_angle;
    d.slot_of_canon = c->upload(c->slot_of_canon);
    d.canon_of_slot = c->upload(canon_of_slot);

    // links in slot space
    std::vector<int> link(2 * (size_t)d.nslots, -1);
    std::vector<unsigned char> fed(2 * (size_t)d.nslots, 0);
    for (int t = 0; t < T; ++t)
        for (int s = 0; s < 2; ++s) {
            const int dst = c->tracks.link[2 * (size_t)t + s];
            if (dst < 0) continue;
            const int t2 = dst / 2, s2 = dst % 2;
            const int j = s2 * d.nslots + c->slot_of_canon[t2];
            link[(size_t)s * d.nslots + c->slot_of_canon[t]] = j;
            fed[j] = 1;
        }
    d.link = c->upload(link);
    d.fed = c->upload(fed);

    // ---- per-region and per-material arrays
    std::vector<int> mat(R);
    for (int r = 0; r < R; ++r) mat[r] = mesh_in->region_material[c->user_of_internal[r]];
    d.mat = c->upload(mat);
    d.user_of = c->upload(c->user_of_internal);
    d.V = c->upload(V_internal);
    d.sigt_m = c->upload(c->sigt_m_host);
    d.sigs_m = c->upload(std::vector<double>(xs->sigma_s, xs->sigma_s + M * G * G));
    d.nsf_m = c->upload(c->nsf_m_host);
    d.chi_m = c->upload(std::vector<double>(xs->chi, xs->chi + M * G));
    // (Sigma_t, qhat) pairs per region and padded group; qhat starts at zero
    if (f64) {
        std::vector<double> xq((size_t)R * d.Gp * 2, 0.0);
        for (int r = 0; r < R; ++r)
            for (int g = 0; g < G; ++g) xq[((size_t)r * d.Gp + g) * 2] = xs->sigma_t[mat[r] * G + g];
        d.xsq = c->upload(xq);
    } else {
        std::vector<float> xq((size_t)R * d.Gp * 2, 0.0f);
        for (int r = 0; r < R; ++r)
            for (int g = 0; g < G; ++g) xq[((size_t)r * d.Gp + g) * 2] = (float)xs->sigma_t[mat[r] * G + g];
        d.xsq = c->upload(xq);
    }
    d.tally = c->dalloc<double>((size_t)R * d.Gp);
    c->tally_rows = c->xsq_rows = R;
    d.phi[0] = c->dalloc<double>((size_t)R * G);
    d.phi[1] = c->dalloc<double>((size_t)R * G);
    const size_t npsi = (size_t)2 * P * d.Gp * d.nslots;
    d.psi[0] = c->dalloc<char>(npsi * rs);
    d.psi[1] = c->dalloc<char>(npsi * rs);
    if (!c->host_only) {
        launch_fill_real(d.psi[0], (int64_t)npsi, d.precision, c->stream);
        launch_fill_real(d.psi[1], (int64_t)npsi, d.precision, c->stream);
    }

    // tally weights c_ap = 2 pi w_a w_p delta_a sin(theta_p); 1/sin(theta_p)
    std::vector<double> coef((size_t)d.NA * P), inv_sin(P);
    for (int a = 0; a < d.NA; ++a)
        for (int p = 0; p < P; ++p)
            coef[(size_t)a * P + p] = 2.0 * 3.14159265358979323846 * c->quad.wa[a] * c->quad.wp[p] * c->quad.delta[a] * c->quad.sinp[p];
    for (int p = 0; p < P; ++p) inv_sin[p] = 1.0 / c->quad.sinp[p];
    if (f64) {
        d.coef = c->upload(coef);
        d.inv_sin = c->upload(inv_sin);
    } else {
        d.coef = c->upload(std::vector<float>(coef.begin(), coef.end()));
        d.inv_sin = c->upload(std::vector<float>(inv_sin.begin(), inv_sin.end()));
    }
    std::vector<float> table(kExpTableN);
    for (int i = 0; i < kExpTableN; ++i) {
        const double x = (double)i * kExpTableMax / kExpTableN;
        table[i] = (float)(i == 0 ? 1.0 : -std::expm1(-x) / x);
    }
    d.exp_table = c->upload(table);
    d.partials = c->dalloc<double>(2 * kReduceBlocks);
    d.scal = c->dalloc<double>(kScalCount);
    d.tally_bound = c->dalloc<unsigned>((size_t)d.Gp);
    if (!c->host_only) {
        launch_fill_f64(d.scal, kScalCount, 0.0, c->stream);
        launch_fill_f64(d.scal, 1, 1.0, c->stream);  // k = 1
        launch_fill_f64(d.phi[0], (int64_t)R * G, 1.0, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static hipStream_t pick(moc_ctx *c, void *s) { return s ? (hipStream_t)s : c->stream; }

static void need_device(const moc_ctx *c) {
    if (c->host_only) throw Error(MOC_ESTATE, "host-only context (negative device ordinal): no device state");
}

static std::pair<hipEvent_t, hipEvent_t> prof_events(moc_ctx *c) {
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

static void sweep_impl(moc_ctx *c, hipStream_t s) {
    DevProblem &d = c->d;
    launch_fill_f64(d.tally, c->tally_rows * d.Gp, 0.0, s);
    SweepArgs a{};
    a.segs = d.segs;
    a.batch_win = d.batch_win;
    a.win_entry_off = d.win_entry_off;
    a.win_nsteps = d.win_nsteps;
    a.win_tab_off = d.win_tab_off;
    a.win_nslots = d.win_nslots;
    a.win_tab = d.win_tab;
    a.cap = d.max_slots;
    a.batch_angle = d.batch_angle;
    a.batch_of_block = d.batch_of_block;
    a.xsq = d.xsq;
    a.psi_in = d.psi[c->cur_psi];
    a.psi_out = d.psi[1 - c->cur_psi];
    a.link = d.link;
    a.fed = d.fed;
    a.coef = d.coef;
    a.inv_sin = d.inv_sin;
    a.exp_table = d.exp_table;
    a.tally = d.tally;
    a.tally_bound = d.tally_bound;
    a.exit_canon = c->exit_canon;
    a.canon_of_slot = d.canon_of_slot;
    a.nslots = d.nslots;
    a.Gp = d.Gp;
    a.G = d.G;
    a.n_real = d.R;
    // the FP32 sweep's window sums are fixed point scaled from a bound of the fluxes
    if (d.precision == MOC_PREC_F32) launch_tally_bound(d, a.psi_in, s);
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->profiling) {
        ev = prof_events(c);
        HIP_OK(hipEventRecord(ev.first, s));
    }
    launch_sweep(a, d.precision, d.exp_mode, c->cmfd, d.nb, d.P, d.gb, d.n_gb, s);
    if (c->profiling) {
        HIP_OK(hipEventRecord(ev.second, s));
        c->prof_pending.push_back(ev);
    }
    c->cur_psi = 1 - c->cur_psi;
}

extern "C" {

int moc_create(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs, const moc_options *opts, moc_ctx **out) {
    if (!out) {
        g_create_error = "create: null output pointer";
        return MOC_EINVAL;
    }
    *out = nullptr;
    moc_ctx *c = new (std::nothrow) moc_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return MOC_ENOMEM;
    }
    const int rc = guarded(c, [&] { create_context(mesh, tracks, xs, opts, c); });
    if (rc != MOC_OK) {
        g_create_error = c->err;
        delete c;
        return rc;
    }
    g_create_error.clear();
    *out = c;
    return MOC_OK;
}

void moc_destroy(moc_ctx *ctx) { delete ctx; }

int moc_sweep(moc_ctx *c, const double *source_dev, double *phi_out_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!source_dev || !phi_out_dev) throw Error(MOC_EINVAL, "sweep: null pointer");
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        hipStream_t s = pick(c, stream);
        launch_prep_user(c->d, source_dev, s);
        sweep_impl(c, s);
        launch_finalize(c->d, nullptr, phi_out_dev, nullptr, s);
    });
}

// Power (eigen) or source (fixed-source) iteration; see moc_solve in moc.h.
static int solve_impl(moc_ctx *c, double tol, int max_iter, int check_every, moc_result *out) {
    if (!out) throw Error(MOC_EINVAL, "solve: null result");
    need_device(c);
    HIP_OK(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    DevProblem &d = c->d;
    hipStream_t s = c->stream;
    const bool eigen = c->fissile && !c->fixed_source;
    const int64_t nphi = (int64_t)d.R * d.G;
    const int64_t npsi = (int64_t)2 * d.P * d.Gp * d.nslots;
    const size_t psi_bytes = (size_t)npsi * (d.precision == MOC_PREC_F64 ? sizeof(double) : sizeof(float));
    int flags = c->fixed_source ? MOC_FLAG_FIXED_SOURCE : 0;
    bool use_guess = false;
    if (c->guess_pending) {
        c->guess_pending = false;
        launch_check_guess(c->guess_phi, nphi, d.partials, s);
        double chk[2];
        HIP_OK(hipMemcpyAsync(chk, d.partials, sizeof chk, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        use_guess = chk[0] == 0.0 && chk[1] > 0.0 && std::isfinite(c->guess_k);
        if (!use_guess) flags |= MOC_FLAG_FELL_BACK_TO_COLD;
    }
    int sweeps = 0;
    double res = 1.0, dk = 1.0, k = 1.0;

    // initial state: the guess (scalar flux, k, boundary fluxes given or made consistent
    // with it by sweeps at a frozen source), or the cold start phi = 1, k = 1, psi = 0;
    // then the normalisation sum V nuSigma_f phi = 1 in eigenvalue mode
    auto start = [&](bool warm) {
        c->cur_phi = 0;
        double k0 = 1.0;
        if (warm) {
            HIP_OK(hipMemcpyAsync(d.phi[0], c->guess_phi, nphi * sizeof(double), hipMemcpyDeviceToDevice, s));
            k0 = c->guess_k;
            if (c->guess_has_psi)
                HIP_OK(hipMemcpyAsync(d.psi[c->cur_psi], c->guess_psi, psi_bytes, hipMemcpyDeviceToDevice, s));
            else
                launch_psi_from_phi(d, d.phi[0], d.psi[c->cur_psi], s);
        } else {
            launch_fill_f64(d.phi[0], nphi, 1.0, s);
            launch_fill_real(d.psi[0], npsi, d.precision, s);
            launch_fill_real(d.psi[1], npsi, d.precision, s);
        }
        c->host_scal[0] = eigen ? (k0 > 0 ? k0 : 1.0) : 1.0;
        HIP_OK(hipMemcpyAsync(d.scal + kScalK, c->host_scal, sizeof(double), hipMemcpyHostToDevice, s));
        if (warm && eigen && !(k0 > 0)) launch_k_estimate(d, d.phi[0], d.partials, s);
        if (warm && !c->guess_has_psi) {
            // boundary fluxes consistent with the guess: sweeps with the source frozen at
            // (phi0, k0); the scalar flux of these sweeps is discarded
            launch_source(d, d.phi[0], s);
            for (int i = 0; i < kWarmBoundarySweeps; ++i) {
                sweep_impl(c, s);
                ++sweeps;
            }
        }
        if (eigen) {
            launch_fission_partials(d, d.phi[0], d.partials, s);
            launch_eigen_update(d, d.partials, 0, s);
            launch_scale_f64(d.phi[0], nphi, d.scal + kScalF, s);
            launch_scale_real(d.psi[c->cur_psi], npsi, d.precision, d.scal + kScalF, s);
        }
        launch_fill_f64(d.scal + kScalRes, 2, 1.0, s);   // no residual or dk yet (the CMFD step reads them)
    };
    // one iteration: source, sweep, scalar flux, (CMFD step), eigenvalue update,
    // normalisation and residual
    auto iterate = [&] {
        double *phi_old = d.phi[c->cur_phi], *phi_new = d.phi[1 - c->cur_phi];
        launch_source(d, phi_old, s);
        sweep_impl(c, s);
        ++sweeps;
        launch_finalize(d, phi_new, nullptr, d.partials, s);
        if (c->cmfd && eigen) {
            // CMFD: coarse eigenvalue and rescaled fine flux / incoming boundary flux
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (c->profiling) {
                ev = prof_events(c);
                HIP_OK(hipEventRecord(ev.first, s));
            }
            launch_cmfd(d, c->cd, phi_new, d.psi[c->cur_psi], s);
            if (c->profiling) {
                HIP_OK(hipEventRecord(ev.second, s));
                c->prof_cmfd_pending.push_back(ev);
            }
            launch_fission_partials(d, phi_new, d.partials, s);
            launch_eigen_update(d, d.partials, 3, s);
        } else {
            launch_eigen_update(d, d.partials, eigen ? 1 : 2, s);
        }
        launch_norm_residual(d, phi_new, phi_old, d.partials, s);
        if (eigen) launch_scale_real(d.psi[c->cur_psi], npsi, d.precision, d.scal + kScalF, s);
        c->cur_phi = 1 - c->cur_phi;
    };
    auto read_back = [&] {
        HIP_OK(hipMemcpyAsync(c->host_scal, d.scal, kScalCount * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        k = c->host_scal[kScalK];
        res = c->host_scal[kScalRes];
        dk = c->host_scal[kScalDk];
        if (!std::isfinite(res) || !std::isfinite(k)) throw Error(MOC_EHIP, "solve: non-finite iterate");
    };

    if (use_guess && !(c->cold_res0 >= 0)) {
        // the cold start's first residual is the bar a guess has to stay under: one cold
        // iteration measures it (once per cross-section set, source mode and coarse mesh)
        start(false);
        iterate();
        read_back();
        c->cold_res0 = res;
    }
    start(use_guess);
    int it = 0;
    bool conv = false;
    for (it = 1; it <= max_iter; ++it) {
        iterate();
        // the first iteration of a warm start also relaxes the guess's boundary fluxes and
        // k, so its residual says little about the guess; the watch starts at the second
        const bool watch = use_guess && it >= 2 && it <= kGuessWatch;
        const bool record = !use_guess && it == 1 && !(c->cold_res0 >= 0);
        if (it % check_every == 0 || it == max_iter || watch || record) {
            read_back();
            if (record) c->cold_res0 = res;
            if (watch && res > c->cold_res0) {
                // the guess does worse than a cold start would: restart cold
                flags |= MOC_FLAG_FELL_BACK_TO_COLD;
                use_guess = false;
                start(false);
                it = 0;
                continue;
            }
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
    out->flags = flags;
    out->sweeps = sweeps;
    out->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return conv ? MOC_OK : MOC_ENOCONV;
}

int moc_solve(moc_ctx *c, double tol, moc_result *out) {
    if (!c) return MOC_EINVAL;
    int status = MOC_OK;
    const int rc = guarded(c, [&] {
        if (!(tol > 0)) throw Error(MOC_EINVAL, "solve: tol must be positive");
        status = solve_impl(c, tol, c->max_iter, c->check_every, out);
    });
    if (rc != MOC_OK) return rc;
    if (status != MOC_OK) c->err = "solve: not converged within max_iter";
    return status;
}

int moc_run_iterations(moc_ctx *c, int n, moc_result *out) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (n <= 0) throw Error(MOC_EINVAL, "run_iterations: n must be positive");
        solve_impl(c, 0.0, n, n, out);
    });
}

int moc_set_initial_guess(moc_ctx *c, const double *phi0_dev, double k0, const double *psi_b0_dev) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!phi0_dev) throw Error(MOC_EINVAL, "initial guess: null phi0");
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        if (!c->guess_phi) c->guess_phi = c->dalloc<double>((size_t)c->d.R * c->d.G);
        launch_permute_rows(c->d, phi0_dev, c->guess_phi, 0, c->stream);
        c->guess_k = k0;
        c->guess_has_psi = psi_b0_dev != nullptr;
        if (psi_b0_dev) {
            const int64_t npsi = (int64_t)2 * c->d.P * c->d.Gp * c->d.nslots;
            if (!c->guess_psi) {
                if (c->d.precision == MOC_PREC_F64)
                    c->guess_psi = c->dalloc<double>((size_t)npsi);
                else
                    c->guess_psi = c->dalloc<float>((size_t)npsi);
            }
            launch_fill_real(c->guess_psi, npsi, c->d.precision, c->stream);
            launch_psi_canon(c->d, const_cast<double *>(psi_b0_dev), c->guess_psi, 0, c->stream);
        }
        HIP_OK(hipStreamSynchronize(c->stream));
        c->guess_pending = true;
    });
}

int moc_get_flux(moc_ctx *c, double *phi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!phi_dev) throw Error(MOC_EINVAL, "get_flux: null pointer");
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        launch_permute_rows(c->d, c->d.phi[c->cur_phi], phi_dev, 1, pick(c, stream));
    });
}

int moc_get_boundary_flux(moc_ctx *c, double *psi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!psi_dev) throw Error(MOC_EINVAL, "get_boundary_flux: null pointer");
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        launch_psi_canon(c->d, psi_dev, c->d.psi[c->cur_psi], 1, pick(c, stream));
    });
}

int moc_set_boundary_flux(moc_ctx *c, const double *psi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!psi_dev) throw Error(MOC_EINVAL, "set_boundary_flux: null pointer");
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        launch_psi_canon(c->d, const_cast<double *>(psi_dev), c->d.psi[c->cur_psi], 0, pick(c, stream));
    });
}

int moc_set_exit_flux_buffer(moc_ctx *c, double *psi_exit_dev) {
    if (!c) return MOC_EINVAL;
    if (c->host_only) return MOC_ESTATE;
    c->exit_canon = psi_exit_dev;
    return MOC_OK;
}

int moc_set_external_source(moc_ctx *c, const double *q_dev) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        need_device(c);
        HIP_OK(hipSetDevice(c->device));
        c->cold_res0 = -1.0;
        if (!q_dev) {
            c->fixed_source = false;
            c->d.qext = nullptr;
            return;
        }
        double *buf = c->d.qext ? c->d.qext : c->dalloc<double>((size_t)c->d.R * c->d.G);
        launch_permute_rows(c->d, q_dev, buf, 0, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
        c->d.qext = buf;
        c->fixed_source = true;
    });
}

int moc_set_materials(moc_ctx *c, const int32_t *region_material, const moc_xs *xs) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        need_device(c);
        DevProblem &d = c->d;
        if (!region_material || !xs || !xs->sigma_t || !xs->sigma_s || !xs->nu_sigma_f || !xs->chi)
            throw Error(MOC_EINVAL, "set_materials: null argument");
        if (xs->n_groups != d.G || xs->n_materials != d.M)
            throw Error(MOC_EINVAL, "set_materials: group and material counts must match the context");
        const int M = d.M, G = d.G, R = d.R;
        for (int i = 0; i < M * G; ++i)
            if (!(xs->sigma_t[i] > 0) || !std::isfinite(xs->sigma_t[i]) || !std::isfinite(xs->nu_sigma_f[i]) ||
                !std::isfinite(xs->chi[i]))
                throw Error(MOC_EINVAL, "set_materials: bad cross sections");
        for (int i = 0; i < M * G * G; ++i)
            if (!std::isfinite(xs->sigma_s[i])) throw Error(MOC_EINVAL, "set_materials: non-finite Sigma_s");
        std::vector<int> mat(R);
        for (int r = 0; r < R; ++r) {
            const int m = region_material[c->user_of_internal[r]];
            if (m < 0 || m >= M) throw Error(MOC_EINVAL, "set_materials: material index out of range");
            mat[r] = m;
        }
        HIP_OK(hipSetDevice(c->device));
        HIP_OK(hipStreamSynchronize(c->stream));
        auto put = [&](void *dst, const void *src, size_t bytes) {
            HIP_OK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        };
        put(d.mat, mat.data(), sizeof(int) * R);
        put(d.sigt_m, xs->sigma_t, sizeof(double) * M * G);
        put(d.sigs_m, xs->sigma_s, sizeof(double) * M * G * G);
        put(d.nsf_m, xs->nu_sigma_f, sizeof(double) * M * G);
        put(d.chi_m, xs->chi, sizeof(double) * M * G);
        if (d.precision == MOC_PREC_F64) {
            std::vector<double> xq((size_t)R * d.Gp * 2, 0.0);
            for (int r = 0; r < R; ++r)
                for (int g = 0; g < G; ++g) xq[((size_t)r * d.Gp + g) * 2] = xs->sigma_t[mat[r] * G + g];
            put(d.xsq, xq.data(), sizeof(double) * xq.size());
        } else {
            std::vector<float> xq((size_t)R * d.Gp * 2, 0.0f);
            for (int r = 0; r < R; ++r)
                for (int g = 0; g < G; ++g) xq[((size_t)r * d.Gp + g) * 2] = (float)xs->sigma_t[mat[r] * G + g];
            put(d.xsq, xq.data(), sizeof(float) * xq.size());
        }
        c->sigt_m_host.assign(xs->sigma_t, xs->sigma_t + M * G);
        c->nsf_m_host.assign(xs->nu_sigma_f, xs->nu_sigma_f + M * G);
        c->fissile = false;
        for (int i = 0; i < M * G; ++i) c->fissile |= xs->nu_sigma_f[i] > 0;
        c->fixed_source = false;
        d.qext = nullptr;
        c->guess_pending = false;
        c->cold_res0 = -1.0;
    });
}

static void free_coarse(moc_ctx *c) {
    DevCoarse &cd = c->cd;
    for (void *p : {(void *)cd.cell_of, (void *)cd.cell_reg_off, (void *)cd.cell_reg, (void *)cd.entry_cell,
                    (void *)cd.adj_off, (void *)cd.adj_surf, (void *)cd.adj_nbr, (void *)cd.adj_sign, (void *)cd.adj_L,
                    (void *)cd.adj_h, (void *)cd.adj_hn, (void *)cd.hsum, (void *)cd.Bs, (void *)cd.Binv, (void *)cd.Aoff,
                    (void *)cd.phih, (void *)cd.Dc, (void *)cd.Ldiag, (void *)cd.fchi, (void *)cd.fnsf, (void *)cd.vec,
                    (void *)cd.ratio, (void *)cd.stats, (void *)cd.piv, (void *)cd.red})
        c->dfree(p);
    cd = DevCoarse();
}

// Coarse mesh for CMFD: surfaces from the tracks, a re-packed segment stream with crossing
// entries, one tally row (and a Sigma_t = 1e30, qhat = 0 row) per surface, the coarse
// geometry for the diffusion couplings and the solver's device arrays.
static void set_coarse_impl(moc_ctx *c, int n_cells, const int32_t *region_cell, const moc_cmfd_options *opts) {
    const auto t0 = std::chrono::steady_clock::now();
    DevProblem &d = c->d;
    const int R = d.R, G = d.G;
    if (!c->host_only) {
        HIP_OK(hipSetDevice(c->device));
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    if (n_cells <= 0 || !region_cell) {
        if (c->cmfd) {
            PackOutput pk;
            pack_and_upload(c, nullptr, pk);
        }
        c->cmfd = false;
        free_coarse(c);
        c->cs = CoarseSurfaces();
        return;
    }
    moc_cmfd_options o{};
    if (opts) o = *opts;
    if (o.tol < 0 || o.max_outer < 0 || o.max_inner < 0) throw Error(MOC_EINVAL, "coarse mesh: negative option");
    if (o.coarse_blocks < 0 || o.coarse_blocks > 256) throw Error(MOC_EINVAL, "coarse mesh: coarse_blocks must be in 0..256");
    if (d.precision == MOC_PREC_F32 && d.exp_mode != MOC_EXP_POLY && d.exp_mode != MOC_EXP_DIFF)
        throw Error(MOC_EINVAL, "coarse mesh: CMFD currents need exp_mode MOC_EXP_POLY or MOC_EXP_DIFF");
    std::vector<int64_t> count(n_cells, 0);
    for (int u = 0; u < R; ++u) {
        if (region_cell[u] < 0 || region_cell[u] >= n_cells) throw Error(MOC_EINVAL, "coarse mesh: cell index out of range");
        ++count[region_cell[u]];
    }
    for (int k = 0; k < n_cells; ++k)
        if (count[k] == 0) throw Error(MOC_EINVAL, "coarse mesh: cell " + std::to_string(k) + " holds no region");
    free_coarse(c);
    CoarseSurfaces &cs = c->cs;
    cs = CoarseSurfaces();
    cs.n_cells = n_cells;
    cs.cell_of.resize(R);
    for (int r = 0; r < R; ++r) cs.cell_of[r] = region_cell[c->user_of_internal[r]];
    find_coarse_surfaces(c->mesh, c->quad, c->tracks, c->internal_of_user.data(), c->n_threads, cs);
    const int Ns = (int)cs.a.size();
    if ((int64_t)R + Ns >= (int64_t(1) << (32 - kSlotBits)))
        throw Error(MOC_EINVAL, "coarse mesh: too many regions plus surfaces for the packed segment key");
    PackOutput pk;
    pack_and_upload(c, &cs, pk);

    // tally and (Sigma_t, qhat) rows of the surfaces
    const int64_t rows = (int64_t)R + Ns;
    const size_t rs = d.precision == MOC_PREC_F64 ? sizeof(double) : sizeof(float);
    if (!c->host_only) {
        if (rows > c->xsq_rows) {
            void *nx = c->dalloc<char>((size_t)rows * d.Gp * 2 * rs);
            HIP_OK(hipMemcpy(nx, d.xsq, (size_t)R * d.Gp * 2 * rs, hipMemcpyDeviceToDevice));
            c->dfree(d.xsq);
            d.xsq = nx;
            c->xsq_rows = rows;
        }
        if (d.precision == MOC_PREC_F64) {
            std::vector<double> xq((size_t)Ns * d.Gp * 2, 0.0);
            for (size_t i = 0; i < xq.size(); i += 2) xq[i] = 1e30;
            if (Ns) HIP_OK(hipMemcpy((double *)d.xsq + (size_t)R * d.Gp * 2, xq.data(), xq.size() * rs, hipMemcpyHostToDevice));
        } else {
            std::vector<float> xq((size_t)Ns * d.Gp * 2, 0.0f);
            for (size_t i = 0; i < xq.size(); i += 2) xq[i] = 1e30f;
            if (Ns) HIP_OK(hipMemcpy((float *)d.xsq + (size_t)R * d.Gp * 2, xq.data(), xq.size() * rs, hipMemcpyHostToDevice));
        }
        if (rows > c->tally_rows) {
            c->dfree(d.tally);
            d.tally = c->dalloc<double>((size_t)rows * d.Gp);
            c->tally_rows = rows;
        }
    }

    // geometry: cell centroids (area weighted), shared edge length and midpoint per surface
    const Mesh &m = c->mesh;
    std::vector<double> carea(n_cells, 0.0), cx(n_cells, 0.0), cy(n_cells, 0.0);
    for (int t = 0; t < m.nt; ++t) {
        const int *v = &m.tri[3 * (size_t)t];
        const double *a = &m.xy[2 * (size_t)v[0]], *b = &m.xy[2 * (size_t)v[1]], *q = &m.xy[2 * (size_t)v[2]];
        const double ar = 0.5 * std::fabs((b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0]));
        const int k = region_cell[m.tri_region[t]];
        carea[k] += ar;
        cx[k] += ar * (a[0] + b[0] + q[0]) / 3.0;
        cy[k] += ar * (a[1] + b[1] + q[1]) / 3.0;
    }
    for (int k = 0; k < n_cells; ++k) {
        cx[k] /= carea[k];
        cy[k] /= carea[k];
    }
    std::vector<double> sL(Ns, 0.0), smx(Ns, 0.0), smy(Ns, 0.0);
    for (size_t h = 0; h < m.twin.size(); ++h) {
        const int tw = m.twin[h];
        if (tw < 0 || (int)h > tw) continue;
        const int ka = region_cell[m.tri_region[h / 3]], kb = region_cell[m.tri_region[tw / 3]];
        if (ka == kb) continue;
        const int id = cs.find(std::min(ka, kb), std::max(ka, kb));
        if (id < 0) continue;   // an edge no track crosses
        const int e = (int)(h % 3);
        const double *p = &m.xy[2 * (size_t)m.tri[h]];
        const double *q = &m.xy[2 * (size_t)m.tri[h - e + (e + 1) % 3]];
        const double len = std::hypot(q[0] - p[0], q[1] - p[1]);
        sL[id] += len;
        smx[id] += len * 0.5 * (p[0] + q[0]);
        smy[id] += len * 0.5 * (p[1] + q[1]);
    }
    // adjacency slots per cell
    std::vector<std::vector<int>> slots(n_cells);
    for (int sf = 0; sf < Ns; ++sf) {
        slots[cs.a[sf]].push_back(2 * sf);
        if (cs.b[sf] >= 0) slots[cs.b[sf]].push_back(2 * sf + 1);
    }
    std::vector<int64_t> adj_off(n_cells + 1, 0);
    std::vector<int> adj_surf, adj_nbr;
    std::vector<double> adj_sign, adj_L, adj_h, adj_hn;
    for (int k = 0; k < n_cells; ++k) {
        for (int code : slots[k]) {
            const int sf = code / 2;
            const bool is_a = (code & 1) == 0;
            const int nb = is_a ? cs.b[sf] : cs.a[sf];
            double L = 0, hs = 0, hn = 0;
            if (nb >= 0 && sL[sf] > 0) {
                L = sL[sf];
                const double mx = smx[sf] / L, my = smy[sf] / L;
                hs = std::hypot(cx[k] - mx, cy[k] - my);
                hn = std::hypot(cx[nb] - mx, cy[nb] - my);
            }
            adj_surf.push_back(sf);
            adj_nbr.push_back(nb);
            adj_sign.push_back(is_a ? 1.0 : -1.0);
            adj_L.push_back(L);
            adj_h.push_back(hs);
            adj_hn.push_back(hn);
        }
        adj_off[k + 1] = (int64_t)adj_surf.size();
    }
    // regions of each cell, entry cells of the incoming track-senses
    std::vector<int64_t> reg_off(n_cells + 1, 0);
    for (int r = 0; r < R; ++r) ++reg_off[cs.cell_of[r] + 1];
    for (int k = 0; k < n_cells; ++k) reg_off[k + 1] += reg_off[k];
    std::vector<int> cell_reg(R);
    {
        std::vector<int64_t> pos(reg_off.begin(), reg_off.end() - 1);
        for (int r = 0; r < R; ++r) cell_reg[pos[cs.cell_of[r]]++] = r;
    }
    std::vector<int> entry_cell(pk.entry_region.size(), -1);
    for (size_t i = 0; i < entry_cell.size(); ++i)
        if (pk.entry_region[i] >= 0) entry_cell[i] = cs.cell_of[pk.entry_region[i]];

    DevCoarse &cd = c->cd;
    cd.C = n_cells;
    cd.Ns = Ns;
    cd.nadj = (int)adj_surf.size();
    cd.max_deg = 0;
    for (int k = 0; k < n_cells; ++k) cd.max_deg = std::max(cd.max_deg, (int)(adj_off[k + 1] - adj_off[k]));
    cd.tol = o.tol > 0 ? o.tol : 1e-3;
    cd.shift = o.shift > 0 ? o.shift : (o.shift < 0 ? 0.0 : 0.02);
    cd.max_outer = o.max_outer > 0 ? o.max_outer : 8;
    cd.max_inner = o.max_inner > 0 ? o.max_inner : 200;
    cd.blocks = o.coarse_blocks;
    if (!c->host_only) {
        const size_t N = (size_t)n_cells * G;
        cd.cell_of = c->upload(cs.cell_of);
        cd.cell_reg_off = c->upload(reg_off);
        cd.cell_reg = c->upload(cell_reg);
        cd.entry_cell = c->upload(entry_cell);
        cd.adj_off = c->upload(adj_off);
        cd.adj_surf = c->upload(adj_surf);
        cd.adj_nbr = c->upload(adj_nbr);
        cd.adj_sign = c->upload(adj_sign);
        cd.adj_L = c->upload(adj_L);
        cd.adj_h = c->upload(adj_h);
        cd.adj_hn = c->upload(adj_hn);
        cd.hsum = c->dalloc<double>((size_t)n_cells * (2 + 4 * G + G * G));
        cd.Bs = c->dalloc<double>(N * G);
        cd.Binv = c->dalloc<double>(N * G);
        cd.Aoff = c->dalloc<double>((size_t)std::max(1, cd.nadj) * G);
        cd.phih = c->dalloc<double>(N);
        cd.Dc = c->dalloc<double>(N);
        cd.Ldiag = c->dalloc<double>(N);
        cd.fchi = c->dalloc<double>(N);
        cd.fnsf = c->dalloc<double>(N);
        cd.vec = c->dalloc<double>((size_t)kCmfdVectors * N);
        cd.ratio = c->dalloc<double>(N);
        cd.stats = c->dalloc<double>(4);
        cd.piv = c->dalloc<int>(N);
        cd.red = c->dalloc<double>(kCmfdRedDoubles);
        int coop = 0;
        HIP_OK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device));
        cd.grid_ok = coop != 0;
        launch_fill_f64(cd.stats, 4, 0.0, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    c->cmfd = true;
    c->coarse_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int moc_set_coarse_mesh(moc_ctx *c, int32_t n_cells, const int32_t *region_cell, const moc_cmfd_options *opts) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        c->cold_res0 = -1.0;
        set_coarse_impl(c, n_cells, region_cell, opts);
    });
}

int moc_get_coarse_info(moc_ctx *c, moc_coarse_info *info) {
    if (!c || !info) return MOC_EINVAL;
    return guarded(c, [&] {
        *info = moc_coarse_info{};
        if (!c->cmfd) return;
        info->n_cells = c->cd.C;
        info->n_surfaces = c->cd.Ns;
        info->n_crossings = c->crossings;
        info->setup_ms = c->coarse_setup_ms;
        if (!c->host_only) {
            double st[4];
            HIP_OK(hipSetDevice(c->device));
            HIP_OK(hipMemcpyAsync(st, c->cd.stats, sizeof st, hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            info->last_outer = (int32_t)st[0];
            info->last_inner = (int32_t)st[1];
            info->last_k = st[2];
        }
    });
}

int moc_get_surface_currents(moc_ctx *c, int32_t *cells, double *current) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!c->cmfd) throw Error(MOC_ESTATE, "surface currents: no coarse mesh set");
        const int Ns = (int)c->cs.a.size(), G = c->d.G, Gp = c->d.Gp;
        if (cells)
            for (int sf = 0; sf < Ns; ++sf) {
                cells[2 * (size_t)sf] = c->cs.a[sf];
                cells[2 * (size_t)sf + 1] = c->cs.b[sf];
            }
        if (current) {
            need_device(c);
            HIP_OK(hipSetDevice(c->device));
            std::vector<double> rows((size_t)Ns * Gp);
            if (Ns)
                HIP_OK(hipMemcpyAsync(rows.data(), c->d.tally + (size_t)c->d.R * Gp, rows.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            for (int sf = 0; sf < Ns; ++sf)
                for (int g = 0; g < G; ++g) current[(size_t)sf * G + g] = rows[(size_t)sf * Gp + g];
        }
    });
}

int moc_locate_points(moc_ctx *c, const double *xy, int64_t n, int32_t *region_out) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        if (!xy || !region_out || n < 0) throw Error(MOC_EINVAL, "locate_points: bad argument");
        const Mesh &m = c->mesh;
        // uniform bucket grid over the bounding box, built on first use
        if (c->loc_nx == 0) {
            const int nb = std::max(1, (int)std::sqrt((double)m.nt / 4.0));
            c->loc_nx = nb;
            c->loc_ny = nb;
            const double W = m.box[2] - m.box[0], H = m.box[3] - m.box[1];
            std::vector<std::vector<int>> cells((size_t)nb * nb);
            for (int t = 0; t < m.nt; ++t) {
                double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
                for (int k = 0; k < 3; ++k)
                    for (int d2 = 0; d2 < 2; ++d2) {
                        const double v = m.xy[2 * (size_t)m.tri[3 * (size_t)t + k] + d2];
                        lo[d2] = std::min(lo[d2], v);
                        hi[d2] = std::max(hi[d2], v);
                    }
                const int i0 = std::max(0, (int)((lo[0] - m.box[0]) / W * nb)), i1 = std::min(nb - 1, (int)((hi[0] - m.box[0]) / W * nb));
                const int j0 = std::max(0, (int)((lo[1] - m.box[1]) / H * nb)), j1 = std::min(nb - 1, (int)((hi[1] - m.box[1]) / H * nb));
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i) cells[(size_t)j * nb + i].push_back(t);
            }
            c->loc_off.assign((size_t)nb * nb + 1, 0);
            for (size_t k = 0; k < cells.size(); ++k) c->loc_off[k + 1] = c->loc_off[k] + (int64_t)cells[k].size();
            c->loc_tri.resize(c->loc_off.back());
            for (size_t k = 0; k < cells.size(); ++k)
                std::copy(cells[k].begin(), cells[k].end(), c->loc_tri.begin() + c->loc_off[k]);
        }
        const double W = m.box[2] - m.box[0], H = m.box[3] - m.box[1];
        for (int64_t q = 0; q < n; ++q) {
            const double px = xy[2 * q], py = xy[2 * q + 1];
            int found = -1;
            const int i = (int)((px - m.box[0]) / W * c->loc_nx), j = (int)((py - m.box[1]) / H * c->loc_ny);
            if (i >= 0 && i < c->loc_nx && j >= 0 && j < c->loc_ny) {
                const size_t cell = (size_t)j * c->loc_nx + i;
                for (int64_t k = c->loc_off[cell]; k < c->loc_off[cell + 1] && found < 0; ++k) {
                    const int t = c->loc_tri[k];
                    const int *v = &m.tri[3 * (size_t)t];
                    bool inside = true;
                    for (int e = 0; e < 3 && inside; ++e) {
                        const double *a = &m.xy[2 * (size_t)v[e]], *b = &m.xy[2 * (size_t)v[(e + 1) % 3]];
                        inside = (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]) >= 0;
                    }
                    if (inside) found = m.tri_region[t];
                }
            }
            region_out[q] = found;
        }
    });
}

int moc_get_centroids(const moc_ctx *c, double *xy_out) {
    if (!c || !xy_out) return MOC_EINVAL;
    const Mesh &m = c->mesh;
    std::vector<double> w(m.R, 0.0);
    for (int r = 0; r < m.R; ++r) xy_out[2 * r] = xy_out[2 * r + 1] = 0.0;
    for (int t = 0; t < m.nt; ++t) {
        const int *v = &m.tri[3 * (size_t)t];
        const double *a = &m.xy[2 * (size_t)v[0]], *b = &m.xy[2 * (size_t)v[1]], *cc = &m.xy[2 * (size_t)v[2]];
        const double ar = 0.5 * ((b[0] - a[0]) * (cc[1] - a[1]) - (b[1] - a[1]) * (cc[0] - a[0]));
        const int r = m.tri_region[t];
        xy_out[2 * r] += ar * (a[0] + b[0] + cc[0]) / 3;
        xy_out[2 * r + 1] += ar * (a[1] + b[1] + cc[1]) / 3;
        w[r] += ar;
    }
    for (int r = 0; r < m.R; ++r) {
        xy_out[2 * r] /= w[r];
        xy_out[2 * r + 1] /= w[r];
    }
    return MOC_OK;
}

int moc_get_info(const moc_ctx *c, moc_info *info) {
    if (!c || !info) return MOC_EINVAL;
    info->n_regions = c->d.R;
    info->n_groups = c->d.G;
    info->n_materials = c->d.M;
    info->n_polar = c->d.P;
    info->n_angles = c->d.NA;
    info->n_tracks = c->d.T;
    info->n_segments = c->S;
    info->n_updates = 2LL * c->d.P * c->d.G * c->S;
    info->n_padded_steps = c->padded_steps;
    info->n_batches = c->d.nb;
    info->n_windows = c->n_windows;
    info->n_window_slots = c->n_slots_total;
    info->window_cm = c->window_len;
    info->max_window_slots = c->d.max_slots;
    info->setup_ms = c->setup_ms;
    info->device_bytes = c->device_bytes;
    info->precision = c->d.precision;
    info->lane_stagger = c->pin.stagger;
    return MOC_OK;
}

static void drain_profile(moc_ctx *c) {
    for (auto &e : c->prof_cmfd_pending) {
        HIP_OK(hipEventSynchronize(e.second));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_cmfd_ms += ms;
        ++c->prof_cmfd_n;
        c->prof_pool.push_back(e);
    }
    c->prof_cmfd_pending.clear();
    for (auto &e : c->prof_pending) {
        HIP_OK(hipEventSynchronize(e.second));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_min = c->prof_n ? std::min(c->prof_min, (double)ms) : ms;
        c->prof_max = c->prof_n ? std::max(c->prof_max, (double)ms) : ms;
        c->prof_ms += ms;
        ++c->prof_n;
        c->prof_pool.push_back(e);
    }
    c->prof_pending.clear();
}

int moc_set_profiling(moc_ctx *c, int enable) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        need_device(c);
        drain_profile(c);
        c->profiling = enable != 0;
        c->prof_n = c->prof_cmfd_n = 0;
        c->prof_ms = c->prof_min = c->prof_max = c->prof_cmfd_ms = 0;
    });
}

int moc_get_profile(moc_ctx *c, moc_profile *out) {
    if (!c || !out) return MOC_EINVAL;
    return guarded(c, [&] {
        need_device(c);
        drain_profile(c);
        out->sweeps = c->prof_n;
        out->sweep_ms = c->prof_ms;
        out->sweep_ms_min = c->prof_min;
        out->sweep_ms_max = c->prof_max;
        out->cmfd_steps = c->prof_cmfd_n;
        out->cmfd_ms = c->prof_cmfd_ms;
    });
}

int moc_get_volumes(const moc_ctx *c, double *V_host) {
    if (!c || !V_host) return MOC_EINVAL;
    std::memcpy(V_host, c->V_user.data(), sizeof(double) * c->V_user.size());
    return MOC_OK;
}

int moc_get_tracks(moc_ctx *c, int32_t *angle, double *endpoints, int64_t *offsets, int32_t *seg_region, double *seg_length,
                   int32_t *links) {
    if (!c) return MOC_EINVAL;
    return guarded(c, [&] {
        const Tracks &t = c->tracks;
        int64_t off = 0;
        for (int i = 0; i < t.T; ++i) {
            if (angle) angle[i] = t.angle[i];
            if (endpoints) {
                endpoints[4 * (size_t)i] = t.x0[i];
                endpoints[4 * (size_t)i + 1] = t.y0[i];
                endpoints[4 * (size_t)i + 2] = t.x1[i];
                endpoints[4 * (size_t)i + 3] = t.y1[i];
            }
            if (links) {
                links[2 * (size_t)i] = t.link[2 * (size_t)i];
                links[2 * (size_t)i + 1] = t.link[2 * (size_t)i + 1];
            }
            if (offsets || seg_region || seg_length) {
                DumpSink ds;
                trace_track(c->mesh, c->quad, t, i, ds);
                if (offsets) offsets[i] = off;
                for (size_t k = 0; k < ds.reg.size(); ++k) {
                    if (seg_region) seg_region[off + (int64_t)k] = ds.reg[k];
                    if (seg_length) seg_length[off + (int64_t)k] = ds.len[k];
                }
                off += (int64_t)ds.reg.size();
            }
        }
        if (offsets) offsets[t.T] = off;
    });
}

int moc_get_packing(const moc_ctx *c, int64_t *batch_win, int32_t *batch_angle, int64_t *win_entry_off,
                    int32_t *win_nsteps, int64_t *win_tab_off, int32_t *win_nslots, int32_t *win_tab,
                    double *seg_len, uint32_t *seg_key, int32_t *user_of_internal) {
    if (!c) return MOC_EINVAL;
    if (!c->host_only) return MOC_ESTATE;
    if (user_of_internal)
        for (int r = 0; r < c->mesh.R; ++r) user_of_internal[r] = c->user_of_internal[r];
    const PackOutput &pk = c->host_pack;
    auto cp = [](auto *dst, const auto &v) {
        if (dst)
            for (size_t i = 0; i < v.size(); ++i) dst[i] = v[i];
    };
    cp(batch_win, pk.batch_win);
    cp(batch_angle, c->host_batch_angle);
    cp(win_entry_off, pk.win_entry_off);
    cp(win_nsteps, pk.win_nsteps);
    cp(win_tab_off, pk.win_tab_off);
    cp(win_nslots, pk.win_nslots);
    cp(win_tab, pk.tab);
    const size_t n = c->d.precision == MOC_PREC_F64 ? c->host_segs_f64.size() : c->host_segs_f32.size();
    for (size_t i = 0; i < n; ++i) {
        if (c->d.precision == MOC_PREC_F64) {
            if (seg_len) seg_len[i] = c->host_segs_f64[i].len;
            if (seg_key) seg_key[i] = c->host_segs_f64[i].key;
        } else {
            if (seg_len) seg_len[i] = c->host_segs_f32[i].len;
            if (seg_key) seg_key[i] = c->host_segs_f32[i].key;
        }
    }
    return MOC_OK;
}

int moc_get_quadrature(const moc_ctx *c, double *phi, double *delta, double *w_azim, double *mu, double *w_polar) {
    if (!c) return MOC_EINVAL;
    for (int a = 0; a < c->quad.NA; ++a) {
        if (phi) phi[a] = c->quad.phi[a];
        if (delta) delta[a] = c->quad.delta[a];
        if (w_azim) w_azim[a] = c->quad.wa[a];
    }
    for (int p = 0; p < c->quad.P; ++p) {
        if (mu) mu[p] = c->quad.mu[p];
        if (w_polar) w_polar[p] = c->quad.wp[p];
    }
    return MOC_OK;
}

const char *moc_last_error(const moc_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

int moc::guarded_call(moc_ctx *c, const std::function<void()> &f) { return guarded(c, f); }
