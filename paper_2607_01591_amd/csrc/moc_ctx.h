// Host-side context of libmoc: the planar problem's geometry, tracks, packing and device
// state (shared by the C ABI of the planar solver and of the extruded DGMOC solver).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "moc_kernels.h"
#include "moc_pack.h"

#define HIP_OK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) throw moc::Error(MOC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct moc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    moc::Mesh mesh;
    moc::Quadrature quad;
    moc::Tracks tracks;
    moc::DevProblem d;
    std::vector<int> internal_of_user, user_of_internal;
    std::vector<int> slot_of_canon;
    std::vector<double> V_user;
    std::vector<double> sigt_m_host, nsf_m_host;
    int64_t S = 0, padded_steps = 0, n_windows = 0, n_slots_total = 0;
    double window_len = 0;
    // host-only contexts keep the packed layout for inspection
    moc::PackOutput host_pack;
    std::vector<moc::SegF> host_segs_f32;
    std::vector<moc::SegD> host_segs_f64;
    std::vector<int> host_batch_angle;
    // point-location buckets (moc_locate_points)
    int loc_nx = 0, loc_ny = 0;
    std::vector<int64_t> loc_off;
    std::vector<int> loc_tri;
    int64_t device_bytes = 0;
    double setup_ms = 0;
    int max_iter = 10000, check_every = 1, n_threads = 1;
    bool host_only = false;   // negative device ordinal: tracking only, no device state
    int cur_psi = 0, cur_phi = 0;
    bool fissile = false;
    bool fixed_source = false;
    // initial guess
    bool guess_pending = false;
    double guess_k = 1.0;
    bool guess_has_psi = false;
    double *guess_phi = nullptr;   // internal [R][G]
    void *guess_psi = nullptr;     // internal boundary-flux layout, sweep precision
    // residual of the first iteration from a cold start with the current cross sections,
    // source mode and coarse mesh (negative: not known yet); a warm start must stay below it
    double cold_res0 = -1.0;
    double *exit_canon = nullptr;  // user buffer
    double *host_scal = nullptr;   // pinned
    std::vector<std::pair<void *, size_t>> allocs;
    std::string err;
    // packing parameters kept for re-packing (coarse mesh on/off)
    moc::PackInput pin;
    int64_t crossings = 0;
    // CMFD coarse mesh
    bool cmfd = false;
    moc::CoarseSurfaces cs;
    moc::DevCoarse cd;
    int64_t tally_rows = 0, xsq_rows = 0;
    double coarse_setup_ms = 0;
    // sweep profiling
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_pool, prof_cmfd_pending;
    int64_t prof_n = 0, prof_cmfd_n = 0;
    double prof_ms = 0, prof_min = 0, prof_max = 0, prof_cmfd_ms = 0;

    template <typename T> T *dalloc(size_t n) {
        if (host_only) return nullptr;
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(n * sizeof(T), 16);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) throw moc::Error(MOC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
        allocs.push_back({p, bytes});
        device_bytes += (int64_t)bytes;
        return (T *)p;
    }
    void dfree(void *p) {
        if (!p) return;
        for (size_t i = 0; i < allocs.size(); ++i)
            if (allocs[i].first == p) {
                if (stream) hipStreamSynchronize(stream);
                hipFree(p);
                device_bytes -= (int64_t)allocs[i].second;
                allocs.erase(allocs.begin() + (long)i);
                return;
            }
    }
    template <typename T> T *upload(const std::vector<T> &v) {
        if (host_only) return nullptr;
        T *p = dalloc<T>(v.size());
        if (!v.empty()) HIP_OK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    ~moc_ctx() {
        if (stream) hipStreamSynchronize(stream);
        for (auto *v : {&prof_pending, &prof_cmfd_pending})
            for (auto &e : *v) {
                hipEventSynchronize(e.second);
                hipEventDestroy(e.first);
                hipEventDestroy(e.second);
            }
        for (auto &e : prof_pool) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
        for (auto &a : allocs) hipFree(a.first);
        if (host_scal) hipHostFree(host_scal);
        if (stream) hipStreamDestroy(stream);
    }
};

namespace moc {
// Host setup of a context: cross sections, mesh, tracks, packing and the planar device
// state (moc_api.cpp). Throws moc::Error.
void create_context(const moc_mesh *mesh, const moc_tracks *tracks, const moc_xs *xs, const moc_options *opt,
                    moc_ctx *c);
// Run f, turning exceptions into status codes and recording the message in c->err.
int guarded_call(moc_ctx *c, const std::function<void()> &f);
}  // namespace moc
