// Packing of traced tracks into 64-track batches and LDS tally windows (moc_pack.cpp).
#pragma once

#include <unordered_map>

#include "moc_internal.h"

namespace moc {

// low bits of a segment key hold the window-local tally slot
constexpr int kSlotBits = 9;
// most entries of one tally window that may fall on one slot: the FP32 sweep's 64-bit
// fixed-point window sums (terms below 2^50) stay below 2^62 up to this count; a window
// above it is split
constexpr int kMaxSlotVisits = 4095;

struct SegF {
    float len;
    uint32_t key;   // (internal region << kSlotBits) | slot
};
struct alignas(16) SegD {
    double len;
    uint32_t key;
    uint32_t pad;
};

// Coarse-cell surfaces crossed by the tracks (CMFD currents). Surface ids are dense:
// interior surfaces are unordered cell pairs (a < b), boundary surfaces are (a, -1).
struct CoarseSurfaces {
    int n_cells = 0;
    std::vector<int> cell_of;            // [R] internal region -> coarse cell
    std::vector<int> a, b;               // [Ns] cells of each surface, b = -1 on the boundary
    std::unordered_map<int64_t, int> id; // pair key -> surface id
    int64_t key(int x, int y) const { return (int64_t)(x + 1) * (n_cells + 1) + (y + 1); }
    int find(int x, int y) const {
        auto it = id.find(key(x, y));
        return it == id.end() ? -1 : it->second;
    }
};

// Trace every track once and collect the coarse surfaces its segments cross.
void find_coarse_surfaces(const Mesh &mesh, const Quadrature &quad, const Tracks &tracks,
                          const int *internal_of_user, int n_threads, CoarseSurfaces &cs);

struct PackInput {
    const Mesh *mesh = nullptr;
    const Quadrature *quad = nullptr;
    const Tracks *tracks = nullptr;
    const int *internal_of_user = nullptr;
    std::vector<int> batch_first;   // [nb + 1] first canonical track of each batch
    double window_len = 1.0;        // cm
    int window_steps = 0;           // > 0: windows of this many steps per lane instead of window_len
    int stagger = 1;                // lane l of a window starts (l mod stagger) steps late
    int cap = 256;                  // maximum tally slots per window
    int n_threads = 1;
    // optional: insert a crossing entry wherever a track enters or leaves a coarse cell;
    // its key holds region n_real + surface id and its length is +1 (sense 0 crosses in
    // the surface's positive orientation: from a to b, or out of the domain) or -1
    const CoarseSurfaces *coarse = nullptr;
};

struct PackOutput {
    int64_t S = 0;                   // real segments
    int64_t crossings = 0;           // coarse-surface crossing entries
    int64_t entries = 0;             // padded entries (steps * 64)
    std::vector<int64_t> batch_win;  // [nb + 1] window range of each batch
    std::vector<int64_t> win_entry_off, win_tab_off;
    std::vector<int> win_nsteps, win_nslots;
    std::vector<int> tab;            // window slot -> internal region
    std::vector<int> entry_region;   // [2][nslots] internal region entered first per track-sense
    std::vector<double> V;           // internal order
};

void pack_segments_f32(const PackInput &in, PackOutput &out, std::vector<SegF> &segs);
void pack_segments_f64(const PackInput &in, PackOutput &out, std::vector<SegD> &segs);

}  // namespace moc
