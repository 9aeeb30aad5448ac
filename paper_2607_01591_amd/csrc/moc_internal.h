// Internal declarations shared by the host setup, the kernels and the C ABI of libmoc.
#pragma once

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "moc.h"

namespace moc {

// Tracks per sweep batch: one wavefront walks 64 adjacent parallel tracks in lockstep.
constexpr int kBatch = 64;
constexpr int kMaxPolar = 4;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// ---------------------------------------------------------------- host geometry
struct Mesh {
    int nv = 0, nt = 0, R = 0;
    std::vector<double> xy;          // [nv][2]
    std::vector<int> tri;            // [nt][3] CCW
    std::vector<int> tri_region;     // [nt] user region id
    std::vector<int> twin;           // [3 nt] half-edge twin, -1 on the boundary
    int domain = MOC_DOMAIN_BOX;
    double box[4] = {0, 0, 0, 0};
    double hex_apothem = 0;
    int bc[6] = {0, 0, 0, 0, 0, 0};
    int n_sides = 4;
    // boundary half-edges per domain side, sorted by their start parameter along the side
    std::vector<std::vector<std::pair<double, int>>> side_edges;
};

struct Quadrature {
    int A = 0, NA = 0, P = 0;
    std::vector<double> phi, delta, wa;  // per track angle (NA)
    std::vector<int> nx, ny;
    std::vector<double> mu, wp, sinp;    // per polar angle
};

struct Tracks {
    int T = 0;
    std::vector<int> angle;              // canonical order
    std::vector<double> x0, y0, x1, y1, len;
    std::vector<int> entry_side;         // side where sense 0 enters
    std::vector<int> link;               // [T][2] destination track*2+sense or -1
};

// setup steps (moc_setup.cpp)
void build_mesh(const moc_mesh &in, Mesh &m);
void build_quadrature(const Mesh &m, const moc_tracks &tr, Quadrature &q);
void lay_tracks(const Mesh &m, const Quadrature &q, Tracks &t);
void link_tracks(const Mesh &m, const Quadrature &q, Tracks &t);

// Walk track t through the mesh (sense 0 order) and call emit(region, length) for each
// merged segment (pieces shorter than 1e-12 cm are dropped, then same-region runs
// merged). Returns the number of segments.
struct SegmentSink {
    virtual void emit(int region, double length) = 0;
    virtual ~SegmentSink() = default;
};
int64_t trace_track(const Mesh &m, const Quadrature &q, const Tracks &t, int track, SegmentSink &sink);

// Morton order of region centroids: internal[user] and user[internal].
void locality_order(const Mesh &m, std::vector<int> &internal_of_user, std::vector<int> &user_of_internal);

// Run f(i) for i in [0, n) on nthreads host threads (dynamic chunks).
void parallel_for(int64_t n, int nthreads, int64_t chunk, const std::function<void(int64_t, int64_t, int)> &f);

}  // namespace moc
