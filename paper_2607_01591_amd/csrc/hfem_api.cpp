// C ABI of libmoc's diffusion HFEM solver (declared in include/hfem.h): host checks of the
// grid and data, the colour ordering and neighbour table of the red-black sweep, the
// device preassembly (Sec. 3.1: matrix construction and two batched inversions per node
// and group), and the power / source iteration of source update, red-black sweeps and
// flux reconstruction. No exception crosses the ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "hfem.h"
#include "hfem_kernels.h"
#include "moc_internal.h"

using namespace moc;

#define HF_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) throw Error(MOC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct moc_hfem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevHF d;
    int nx = 0, ny = 0, nz = 0;
    int nv = 2, nf = 1, n_inner = 2;
    int max_iter = 10000, check_every = 1;
    bool fissile = false, fixed_source = false;
    bool host_only = false;
    int cur_phi = 0;
    double setup_ms = 0, assemble_ms = 0;
    int64_t device_bytes = 0;
    double *host_scal = nullptr;
    double *qext_store = nullptr;
    std::vector<std::pair<void *, size_t>> allocs;
    std::string err;
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_pool;
    int64_t prof_n = 0;
    double prof_ms = 0, prof_min = 0, prof_max = 0;

    template <typename T> T *dalloc(size_t n) {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(n * sizeof(T), 16);
        if (hipMalloc(&p, bytes) != hipSuccess)
            throw Error(MOC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        allocs.push_back({p, bytes});
        device_bytes += (int64_t)bytes;
        return (T *)p;
    }
    template <typename T> T *upload(const std::vector<T> &v) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) HF_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    ~moc_hfem_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
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

static thread_local std::string g_hf_create_error;

static int hf_guarded(moc_hfem_ctx *c, const std::function<void()> &f) {
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

// Legendre degree triples of the volume basis: by total degree, a then b descending
static std::vector<int> hf_volume_modes(int nv) {
    std::vector<int> out;
    for (int n = 0; n <= nv; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                out.push_back(a);
                out.push_back(b);
                out.push_back(n - a - b);
            }
    return out;
}

// degree pairs of a face basis: by total degree, first degree descending
static std::vector<int> hf_face_modes(int nf) {
    std::vector<int> out;
    for (int t = 0; t <= nf; ++t)
        for (int m = t; m >= 0; --m) {
            out.push_back(m);
            out.push_back(t - m);
        }
    return out;
}

static void hf_check_edges(const double *e, int n, const char *name) {
    if (n <= 0 || !e) throw Error(MOC_EINVAL, std::string("grid: no ") + name + " edges");
    for (int i = 0; i <= n; ++i)
        if (!std::isfinite(e[i])) throw Error(MOC_EINVAL, std::string("grid: non-finite ") + name + " edge");
    for (int i = 0; i < n; ++i)
        if (!(e[i + 1] > e[i])) throw Error(MOC_EINVAL, std::string("grid: ") + name + " edges not strictly increasing");
}

static void hf_create_impl(const moc_hfem_grid *grid, const moc_xs *xs, const moc_hfem_options *opt, moc_hfem_ctx *c) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!grid || !xs) throw Error(MOC_EINVAL, "hfem create: null argument");
    moc_hfem_options o{};
    o.volume_order = 2;
    o.face_order = 1;
    if (opt) o = *opt;
    if (o.volume_order < 0 || o.volume_order > 4) throw Error(MOC_EINVAL, "options: volume_order must be 0..4");
    if (o.face_order < 0 || o.face_order > 2 || o.face_order > o.volume_order)
        throw Error(MOC_EINVAL, "options: face_order must be 0..2 and at most volume_order");
    c->nv = o.volume_order;
    c->nf = o.face_order;
    c->n_inner = o.inner_iterations > 0 ? o.inner_iterations : 2;
    c->max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    c->check_every = o.check_every > 0 ? o.check_every : 1;
    const int nx = grid->nx, ny = grid->ny, nz = grid->nz;
    hf_check_edges(grid->x_edges, nx, "x");
    hf_check_edges(grid->y_edges, ny, "y");
    hf_check_edges(grid->z_edges, nz, "z");
    const int64_t N64 = (int64_t)nx * ny * nz;
    const int M = xs->n_materials, G = xs->n_groups;
    if (M <= 0 || G <= 0 || !xs->sigma_t || !xs->sigma_s || !xs->nu_sigma_f || !xs->chi)
        throw Error(MOC_EINVAL, "xs: empty or null arrays");
    if (N64 * G > (int64_t)1 << 30) throw Error(MOC_EINVAL, "grid: too many node-groups");
    const int N = (int)N64;
    if (!grid->node_material) throw Error(MOC_EINVAL, "grid: null node_material");
    for (int e = 0; e < N; ++e)
        if (grid->node_material[e] < 0 || grid->node_material[e] >= M)
            throw Error(MOC_EINVAL, "grid: material index out of range");
    for (int f = 0; f < 6; ++f)
        if (grid->bc[f] != MOC_BC_VACUUM && grid->bc[f] != MOC_BC_REFLECTIVE)
            throw Error(MOC_EINVAL, "grid: bc must be vacuum (0) or reflective (1)");
    std::vector<double> diff((size_t)M * G), sigr((size_t)M * G);
    for (int m = 0; m < M; ++m)
        for (int g = 0; g < G; ++g) {
            const double st = xs->sigma_t[m * G + g];
            if (!(st > 0) || !std::isfinite(st)) throw Error(MOC_EINVAL, "xs: Sigma_t must be positive and finite");
            const double sr = st - xs->sigma_s[((size_t)m * G + g) * G + g];
            if (!(sr > 0) || !std::isfinite(sr)) throw Error(MOC_EINVAL, "xs: removal Sigma_t - Sigma_s(g->g) must be positive");
            diff[(size_t)m * G + g] = 1.0 / (3.0 * st);
            sigr[(size_t)m * G + g] = sr;
        }
    for (int64_t i = 0; i < (int64_t)M * G * G; ++i)
        if (!std::isfinite(xs->sigma_s[i])) throw Error(MOC_EINVAL, "xs: non-finite Sigma_s");
    for (int i = 0; i < M * G; ++i) {
        if (!std::isfinite(xs->nu_sigma_f[i]) || !std::isfinite(xs->chi[i])) throw Error(MOC_EINVAL, "xs: non-finite data");
        c->fissile |= xs->nu_sigma_f[i] > 0;
    }
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;

    DevHF &d = c->d;
    const std::vector<int> vm = hf_volume_modes(c->nv), fm = hf_face_modes(c->nf);
    d.N = N;
    d.G = G;
    d.M = M;
    d.Np = (int)vm.size() / 3;
    d.Nfb = (int)fm.size() / 2;
    d.Nft = 6 * d.Nfb;

    // ---- colour order (red: i + j + k even, first), neighbours, node sizes and volumes
    std::vector<int> perm, pos(N);
    perm.reserve(N);
    for (int colour = 0; colour < 2; ++colour)
        for (int e = 0; e < N; ++e) {
            const int i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
            if ((i + j + k) % 2 == colour) perm.push_back(e);
        }
    int n_red = 0;
    for (int e = 0; e < N; ++e) {
        const int i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
        n_red += (i + j + k) % 2 == 0;
    }
    d.n_red = n_red;
    for (int p = 0; p < N; ++p) pos[perm[p]] = p;
    std::vector<int> nbr((size_t)N * 6);
    std::vector<double> hdim((size_t)N * 3), vol(N);
    const int dims[3] = {nx, ny, nz};
    const int stride[3] = {1, nx, nx * ny};
    const double *edges[3] = {grid->x_edges, grid->y_edges, grid->z_edges};
    for (int p = 0; p < N; ++p) {
        const int e = perm[p];
        const int ijk[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
        double v = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double h = edges[ax][ijk[ax] + 1] - edges[ax][ijk[ax]];
            hdim[(size_t)p * 3 + ax] = h;
            v *= h;
            for (int side = 0; side < 2; ++side) {
                const int f = 2 * ax + side;
                const bool inside = side == 0 ? ijk[ax] > 0 : ijk[ax] < dims[ax] - 1;
                int code;
                if (inside)
                    code = pos[e + (side == 0 ? -stride[ax] : stride[ax])];
                else
                    code = grid->bc[f] == MOC_BC_REFLECTIVE ? kHfReflect : kHfVacuum;
                nbr[(size_t)p * 6 + f] = code;
            }
        }
        vol[e] = v;
    }
    // the sweep of one colour must read only the other colour's currents
    for (int p = 0; p < N; ++p)
        for (int f = 0; f < 6; ++f) {
            const int q = nbr[(size_t)p * 6 + f];
            if (q >= 0 && ((p < n_red) == (q < n_red))) throw Error(MOC_EINVAL, "internal: neighbours of one colour");
        }

    if (o.device < 0) {
        c->host_only = true;
        c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return;
    }
    c->device = o.device;
    HF_HIP(hipSetDevice(c->device));
    HF_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HF_HIP(hipHostMalloc((void **)&c->host_scal, kHfCount * sizeof(double), hipHostMallocDefault));
    std::vector<int> mat(grid->node_material, grid->node_material + N);
    const int Np = d.Np, Nft = d.Nft;
    const size_t npg = (size_t)N * G;
    d.perm = c->upload(perm);
    d.pos = c->upload(pos);
    d.nbr = c->upload(nbr);
    d.hdim = c->upload(hdim);
    d.mat = c->upload(mat);
    d.vol = c->upload(vol);
    d.diff = c->upload(diff);
    d.sigr = c->upload(sigr);
    d.sigs = c->upload(std::vector<double>(xs->sigma_s, xs->sigma_s + (size_t)M * G * G));
    d.nsf = c->upload(std::vector<double>(xs->nu_sigma_f, xs->nu_sigma_f + (size_t)M * G));
    d.chi = c->upload(std::vector<double>(xs->chi, xs->chi + (size_t)M * G));
    d.vmode = c->upload(vm);
    d.npg_blk = 256 / Nft;
    d.nblk[0] = ((int64_t)n_red * G + d.npg_blk - 1) / d.npg_blk;
    d.nblk[1] = ((int64_t)(N - n_red) * G + d.npg_blk - 1) / d.npg_blk;
    const size_t slots = (size_t)(d.nblk[0] + d.nblk[1]) * d.npg_blk;   // node-groups incl. block padding
    d.mat32 = o.fp32_matrices ? 1 : 0;
    if (d.mat32) {
        d.R = c->dalloc<float>(slots * Nft * Nft);
        d.Ainv = c->dalloc<float>(slots * Np * Np);
    } else {
        d.R = c->dalloc<double>(slots * Nft * Nft);
        d.Ainv = c->dalloc<double>(slots * Np * Np);
    }
    // face factor t of face DoF r and volume mode k: sqrt(2a+1) (+-1)^a for the degree a
    // normal to the face when the transverse degrees match the face mode, else 0
    std::vector<double> tface((size_t)Nft * Np, 0.0);
    for (int r = 0; r < Nft; ++r) {
        const int f = r / d.Nfb, mm = r % d.Nfb, ax = f / 2;
        const int t0 = ax == 0 ? 1 : 0, t1 = ax == 2 ? 1 : 2;
        for (int k = 0; k < Np; ++k) {
            const int *vk = &vm[3 * (size_t)k];
            if (vk[t0] != fm[2 * (size_t)mm] || vk[t1] != fm[2 * (size_t)mm + 1]) continue;
            const double v = std::sqrt(2.0 * vk[ax] + 1.0);
            tface[(size_t)r * Np + k] = (f % 2 == 1 || vk[ax] % 2 == 0) ? v : -v;
        }
    }
    d.tface = c->upload(tface);
    // per moment, the face DoFs it couples to (at most one mode on each of the 6 faces)
    std::vector<int> flist((size_t)Np * 6, -1);
    std::vector<double> fval((size_t)Np * 6, 0.0);
    for (int k = 0; k < Np; ++k) {
        int q = 0;
        for (int r = 0; r < Nft; ++r)
            if (tface[(size_t)r * Np + k] != 0.0) {
                if (q == 6) throw Error(MOC_EINVAL, "internal: a moment couples to more than 6 face DoFs");
                flist[(size_t)k * 6 + q] = r;
                fval[(size_t)k * 6 + q] = tface[(size_t)r * Np + k];
                ++q;
            }
    }
    d.flist = c->upload(flist);
    d.fval = c->upload(fval);
    // per face DoF, the moments it couples to
    d.nr = c->nv + 1;
    std::vector<int> rlist((size_t)Nft * d.nr, -1);
    std::vector<double> rval((size_t)Nft * d.nr, 0.0);
    for (int r = 0; r < Nft; ++r) {
        int q = 0;
        for (int k = 0; k < Np; ++k)
            if (tface[(size_t)r * Np + k] != 0.0) {
                if (q == d.nr) throw Error(MOC_EINVAL, "internal: a face DoF couples to too many moments");
                rlist[(size_t)r * d.nr + q] = k;
                rval[(size_t)r * d.nr + q] = tface[(size_t)r * Np + k];
                ++q;
            }
    }
    d.rlist = c->upload(rlist);
    d.rval = c->upload(rval);
    d.jp = c->dalloc<double>(npg * Nft);
    d.s = c->dalloc<double>(npg * Np);
    d.bq = c->dalloc<double>(npg * Nft);
    d.phi[0] = c->dalloc<double>(npg * Np);
    d.phi[1] = c->dalloc<double>(npg * Np);
    d.partials = c->dalloc<double>(2 * kHfReduceBlocks);
    d.scal = c->dalloc<double>(kHfCount);
    d.status = c->dalloc<int>(1);
    hipStream_t s = c->stream;
    HF_HIP(hipMemsetAsync(d.status, 0, sizeof(int), s));
    HF_HIP(hipStreamSynchronize(s));

    // ---- preassembly (timed on the device)
    hipEvent_t e0, e1;
    HF_HIP(hipEventCreate(&e0));
    HF_HIP(hipEventCreate(&e1));
    HF_HIP(hipEventRecord(e0, s));
    launch_hf_assemble(d, s);
    HF_HIP(hipEventRecord(e1, s));
    HF_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HF_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->assemble_ms = ms;
    int status = 0;
    HF_HIP(hipMemcpy(&status, d.status, sizeof(int), hipMemcpyDeviceToHost));
    if (status) throw Error(MOC_EINVAL, "hfem create: singular matrix in the preassembly");

    launch_hf_fill(d.jp, (int64_t)npg * Nft, 0.0, s);
    launch_hf_fill(d.s, (int64_t)npg * Np, 0.0, s);
    launch_hf_cold(d, d.phi[0], s);
    launch_hf_fill(d.scal, kHfCount, 0.0, s);
    launch_hf_fill(d.scal + kHfK, 1, 1.0, s);
    HF_HIP(hipStreamSynchronize(s));
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static std::pair<hipEvent_t, hipEvent_t> hf_prof_events(moc_hfem_ctx *c) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->prof_pool.empty()) {
        HF_HIP(hipEventCreate(&ev.first));
        HF_HIP(hipEventCreate(&ev.second));
    } else {
        ev = c->prof_pool.back();
        c->prof_pool.pop_back();
    }
    return ev;
}

static void hf_drain_profile(moc_hfem_ctx *c) {
    for (auto &e : c->prof_pending) {
        HF_HIP(hipEventSynchronize(e.second));
        float ms = 0;
        HF_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_ms += ms;
        c->prof_min = c->prof_n == 0 ? ms : std::min(c->prof_min, (double)ms);
        c->prof_max = c->prof_n == 0 ? ms : std::max(c->prof_max, (double)ms);
        ++c->prof_n;
        c->prof_pool.push_back(e);
    }
    c->prof_pending.clear();
}

// One HFEM solve after launch_hf_prepare has formed s and h: the red-black iterations
// (each timed when profiling), then the reconstruction into phi_out.
static void hf_sweep_impl(moc_hfem_ctx *c, double *phi_out, hipStream_t s) {
    DevHF &d = c->d;
    for (int it = 0; it < c->n_inner; ++it) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (c->profiling) {
            ev = hf_prof_events(c);
            HF_HIP(hipEventRecord(ev.first, s));
        }
        launch_hf_rb(d, 0, s);
        launch_hf_rb(d, 1, s);
        if (c->profiling) {
            HF_HIP(hipEventRecord(ev.second, s));
            c->prof_pending.push_back(ev);
        }
    }
    launch_hf_reconstruct(d, phi_out, s);
}

static void hf_need_device(const moc_hfem_ctx *c) {
    if (c->host_only) throw Error(MOC_ESTATE, "host-only context (negative device ordinal): no device state");
}

static int hf_solve_impl(moc_hfem_ctx *c, double tol, int max_iter, int check_every, moc_result *out) {
    if (!out) throw Error(MOC_EINVAL, "hfem solve: null result");
    hf_need_device(c);
    HF_HIP(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    DevHF &d = c->d;
    hipStream_t s = c->stream;
    const bool eigen = c->fissile && !c->fixed_source;
    c->cur_phi = 0;
    launch_hf_cold(d, d.phi[0], s);
    launch_hf_fill(d.jp, (int64_t)d.N * d.G * d.Nft, 0.0, s);
    launch_hf_fill(d.scal, kHfCount, 0.0, s);
    launch_hf_fill(d.scal + kHfK, 1, 1.0, s);
    int it = 0, sweeps = 0;
    bool conv = false;
    double res = 1.0, dk = 1.0, k = 1.0;
    for (it = 1; it <= max_iter; ++it) {
        double *phi_old = d.phi[c->cur_phi], *phi_new = d.phi[1 - c->cur_phi];
        launch_hf_prepare(d, phi_old, nullptr, s);
        hf_sweep_impl(c, phi_new, s);
        ++sweeps;
        launch_hf_fission(d, phi_new, phi_old, s);
        launch_hf_eigen(d, eigen ? 0 : 1, s);
        launch_hf_residual(d, phi_new, phi_old, eigen ? 0 : 1, s);
        c->cur_phi = 1 - c->cur_phi;
        if (it % check_every == 0 || it == max_iter) {
            HF_HIP(hipMemcpyAsync(c->host_scal, d.scal, kHfCount * sizeof(double), hipMemcpyDeviceToHost, s));
            HF_HIP(hipStreamSynchronize(s));
            k = c->host_scal[kHfK];
            res = c->host_scal[kHfRes];
            dk = c->host_scal[kHfDk];
            if (!std::isfinite(res) || !std::isfinite(k)) throw Error(MOC_EHIP, "hfem solve: non-finite iterate");
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

int moc_hfem_create(const moc_hfem_grid *grid, const moc_xs *xs, const moc_hfem_options *opts, moc_hfem_ctx **out) {
    if (!out) {
        g_hf_create_error = "hfem create: null output pointer";
        return MOC_EINVAL;
    }
    *out = nullptr;
    moc_hfem_ctx *c = new (std::nothrow) moc_hfem_ctx();
    if (!c) {
        g_hf_create_error = "host allocation failed";
        return MOC_ENOMEM;
    }
    const int rc = hf_guarded(c, [&] { hf_create_impl(grid, xs, opts, c); });
    if (rc != MOC_OK) {
        g_hf_create_error = c->err;
        delete c;
        return rc;
    }
    g_hf_create_error.clear();
    *out = c;
    return MOC_OK;
}

void moc_hfem_destroy(moc_hfem_ctx *c) { delete c; }

int moc_hfem_sweep(moc_hfem_ctx *c, const double *source_dev, double *phi_out_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        if (!source_dev || !phi_out_dev) throw Error(MOC_EINVAL, "hfem sweep: null pointer");
        hf_need_device(c);
        HF_HIP(hipSetDevice(c->device));
        hipStream_t s = stream ? (hipStream_t)stream : c->stream;
        launch_hf_prepare(c->d, nullptr, source_dev, s);
        hf_sweep_impl(c, phi_out_dev, s);
    });
}

int moc_hfem_solve(moc_hfem_ctx *c, double tol, moc_result *out) {
    if (!c) return MOC_EINVAL;
    int status = MOC_OK;
    const int rc = hf_guarded(c, [&] {
        if (!(tol > 0)) throw Error(MOC_EINVAL, "hfem solve: tol must be positive");
        status = hf_solve_impl(c, tol, c->max_iter, c->check_every, out);
    });
    if (rc != MOC_OK) return rc;
    if (status != MOC_OK) c->err = "hfem solve: not converged within max_iter";
    return status;
}

int moc_hfem_run_iterations(moc_hfem_ctx *c, int32_t n, moc_result *out) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        if (n <= 0) throw Error(MOC_EINVAL, "hfem run_iterations: n must be positive");
        hf_solve_impl(c, 0.0, n, n, out);
    });
}

int moc_hfem_get_flux(moc_hfem_ctx *c, double *phi_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        if (!phi_dev) throw Error(MOC_EINVAL, "hfem get_flux: null pointer");
        hf_need_device(c);
        HF_HIP(hipSetDevice(c->device));
        hipStream_t s = stream ? (hipStream_t)stream : c->stream;
        HF_HIP(hipMemcpyAsync(phi_dev, c->d.phi[c->cur_phi], (size_t)c->d.N * c->d.G * c->d.Np * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    });
}

int moc_hfem_get_currents(moc_hfem_ctx *c, double *jplus_dev, void *stream) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        if (!jplus_dev) throw Error(MOC_EINVAL, "hfem get_currents: null pointer");
        hf_need_device(c);
        HF_HIP(hipSetDevice(c->device));
        hipStream_t s = stream ? (hipStream_t)stream : c->stream;
        launch_hf_currents_to_nodes(c->d, jplus_dev, s);
    });
}

int moc_hfem_set_external_source(moc_hfem_ctx *c, const double *q_dev) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        hf_need_device(c);
        HF_HIP(hipSetDevice(c->device));
        DevHF &d = c->d;
        if (!q_dev) {
            c->fixed_source = false;
            d.qext = nullptr;
            return;
        }
        const size_t n = (size_t)d.N * d.G * d.Np;
        if (!c->qext_store) c->qext_store = c->dalloc<double>(n);   // kept for the context's lifetime
        HF_HIP(hipMemcpyAsync(c->qext_store, q_dev, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HF_HIP(hipStreamSynchronize(c->stream));
        d.qext = c->qext_store;
        c->fixed_source = true;
    });
}

int moc_hfem_get_info(const moc_hfem_ctx *c, moc_hfem_info *info) {
    if (!c || !info) return MOC_EINVAL;
    info->n_nodes = c->d.N;
    info->n_groups = c->d.G;
    info->n_moments = c->d.Np;
    info->n_face_dofs = c->d.Nft;
    info->n_red = c->d.n_red;
    info->n_black = c->d.N - c->d.n_red;
    info->inner_iterations = c->n_inner;
    info->device_bytes = c->device_bytes;
    info->setup_ms = c->setup_ms;
    info->assemble_ms = c->assemble_ms;
    info->fp32_matrices = c->d.mat32;
    return MOC_OK;
}

int moc_hfem_set_profiling(moc_hfem_ctx *c, int32_t enable) {
    if (!c) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        hf_drain_profile(c);
        c->profiling = enable != 0;
        c->prof_n = 0;
        c->prof_ms = c->prof_min = c->prof_max = 0;
    });
}

int moc_hfem_get_profile(moc_hfem_ctx *c, moc_profile *out) {
    if (!c || !out) return MOC_EINVAL;
    return hf_guarded(c, [&] {
        hf_drain_profile(c);
        std::memset(out, 0, sizeof *out);
        out->sweeps = c->prof_n;
        out->sweep_ms = c->prof_ms;
        out->sweep_ms_min = c->prof_min;
        out->sweep_ms_max = c->prof_max;
    });
}

const char *moc_hfem_last_error(const moc_hfem_ctx *c) { return c ? c->err.c_str() : g_hf_create_error.c_str(); }

}  // extern "C"
