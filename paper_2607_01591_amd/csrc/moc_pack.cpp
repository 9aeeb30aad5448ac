// Device packing of the traced segments into sweep batches and tally windows.
//
// A batch is up to 64 adjacent parallel tracks of one angle (one per lane of a
// wavefront). Each batch is cut along the track direction into windows of about
// `window_len` cm: lane l's part of window w holds its segments whose start lies in
// [w L, (w + 1) L). Within a window the lanes advance in lockstep (shorter lanes are
// padded with zero-length steps), and every distinct region the window touches gets a
// window-local tally slot, so the sweep kernel can accumulate the window's tallies in
// LDS and flush each slot once. A window whose slot count exceeds `cap`, or in which
// more than kMaxSlotVisits entries fall on one region, is split in half.
//
// Segment entry: {length, key}, key = (internal region << kSlotBits) | slot.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "moc_pack.h"

namespace moc {

namespace {

struct LaneSeg {
    int reg;      // internal region, or n_real + surface id for a crossing entry
    double len;   // length; +-1 (orientation) for a crossing entry
    double s0;    // distance of the segment start from the track start (sense 0)
};

// Insert the coarse-surface crossing entries into one track's segment list: entering the
// domain, every change of coarse cell, leaving the domain.
void add_crossings(const CoarseSurfaces &cs, int n_real, std::vector<LaneSeg> &v, std::vector<LaneSeg> &tmp) {
    if (v.empty()) return;
    tmp.clear();
    int prev = -1;
    for (size_t k = 0; k < v.size(); ++k) {
        const int c = cs.cell_of[v[k].reg];
        if (k == 0) {
            tmp.push_back({n_real + cs.find(c, -1), -1.0, v[k].s0});          // into the domain
        } else if (c != prev) {
            const int lo = std::min(prev, c), hi = std::max(prev, c);
            tmp.push_back({n_real + cs.find(lo, hi), prev < c ? 1.0 : -1.0, v[k].s0});
        }
        tmp.push_back(v[k]);
        prev = c;
    }
    tmp.push_back({n_real + cs.find(prev, -1), 1.0, v.back().s0 + v.back().len});  // out of the domain
    v.swap(tmp);
}

struct CollectSink : SegmentSink {
    std::vector<LaneSeg> *out = nullptr;
    const int *internal_of_user = nullptr;
    double s = 0;
    void emit(int r, double len) override {
        out->push_back({internal_of_user[r], len, s});
        s += len;
    }
};

struct Window {
    int nsteps = 0, nslots = 0;
    int64_t entry_off = 0, tab_off = 0;   // relative to the batch
    std::array<int, kBatch> count{};       // segments of each lane in this window
};

class BatchPlanner {
  public:
    explicit BatchPlanner(const PackInput &in) : in_(in), lanes_(kBatch), ptr_(kBatch), end_(kBatch) {}

    // trace tracks [t0, t1) (one per lane) and cut them into windows
    void plan(int t0, int t1) {
        CollectSink sink;
        sink.internal_of_user = in_.internal_of_user;
        for (auto &v : lanes_) v.clear();
        for (int t = t0; t < t1; ++t) {
            sink.out = &lanes_[t - t0];
            sink.s = 0;
            trace_track(*in_.mesh, *in_.quad, *in_.tracks, t, sink);
            if (in_.coarse) add_crossings(*in_.coarse, in_.mesh->R, lanes_[t - t0], tmp_);
        }
        windows_.clear();
        tab_.clear();
        steps_ = 0;
        double len = 0;
        for (int l = 0; l < kBatch; ++l) {
            ptr_[l] = 0;
            if (!lanes_[l].empty()) len = std::max(len, lanes_[l].back().s0 + lanes_[l].back().len);
        }
        if (in_.window_steps > 0) {
            size_t nmax = 0;
            for (int l = 0; l < kBatch; ++l) nmax = std::max(nmax, lanes_[l].size());
            const size_t K = (size_t)in_.window_steps;
            for (size_t k0 = 0; k0 < nmax; k0 += K) step_range(k0, std::min(nmax, k0 + K));
            return;
        }
        const int nw = std::max(1, (int)std::ceil(len / in_.window_len));
        for (int w = 0; w < nw; ++w) range(w * in_.window_len, (w + 1) * in_.window_len, w == nw - 1);
    }

    int64_t steps() const { return steps_; }
    int64_t n_windows() const { return (int64_t)windows_.size(); }
    int64_t n_slots() const { return (int64_t)tab_.size(); }
    int64_t n_segments() const {
        int64_t n = 0;
        for (const auto &v : lanes_)
            for (const LaneSeg &s : v) n += s.reg < in_.mesh->R;
        return n;
    }
    int64_t n_entries() const {
        int64_t n = 0;
        for (const auto &v : lanes_) n += (int64_t)v.size();
        return n;
    }
    const std::vector<LaneSeg> &lane(int l) const { return lanes_[l]; }
    const std::vector<Window> &windows() const { return windows_; }
    const std::vector<int> &tab() const { return tab_; }

    template <typename Seg> void write(Seg *segs) const {
        std::array<size_t, kBatch> p{};
        for (const Window &w : windows_) {
            const int *wt = tab_.data() + w.tab_off;
            const uint32_t pad_key = (uint32_t)wt[0] << kSlotBits;
            for (int l = 0; l < kBatch; ++l) {
                const auto &v = lanes_[l];
                const int o = lane_offset(l, w.count[l]);
                for (int j = 0; j < w.nsteps; ++j) {
                    Seg &e = segs[w.entry_off + (int64_t)j * kBatch + l];
                    if (j >= o && j - o < w.count[l]) {
                        const LaneSeg &s = v[p[l] + (j - o)];
                        const int slot = int(std::lower_bound(wt, wt + w.nslots, s.reg) - wt);
                        e.len = (decltype(e.len))s.len;
                        e.key = ((uint32_t)s.reg << kSlotBits) | (uint32_t)slot;
                    } else {
                        e.len = 0;
                        e.key = pad_key;
                    }
                }
                p[l] += w.count[l];
            }
        }
    }

  private:
    // first step of lane l inside a window: staggered so that lanes at one step sit at
    // different places along their tracks (fewer lanes adding to one LDS tally row at once)
    int lane_offset(int l, int count) const { return count > 0 ? l % in_.stagger : 0; }
    int window_steps_of(const std::array<int, kBatch> &count) const {
        int n = 0;
        for (int l = 0; l < kBatch; ++l)
            if (count[l] > 0) n = std::max(n, lane_offset(l, count[l]) + count[l]);
        return n;
    }

    // windows by step index: lane l takes its segments [k0, k1) (no spatial alignment)
    void step_range(size_t k0, size_t k1) {
        for (int l = 0; l < kBatch; ++l) {
            ptr_[l] = std::min(k0, lanes_[l].size());
            end_[l] = std::min(k1, lanes_[l].size());
        }
        emit_or_split([&](int half) {
            const size_t mid = (k0 + k1) / 2;
            if (half == 0) step_range(k0, mid); else step_range(mid, k1);
        });
    }

    // emit the window [ptr_, end_) or, above the slot cap, call split(0) then split(1)
    template <typename F> void emit_or_split(F split) {
        int maxn = 0;
        for (int l = 0; l < kBatch; ++l) maxn = std::max(maxn, int(end_[l] - ptr_[l]));
        if (maxn == 0) return;
        regs_.clear();
        for (int l = 0; l < kBatch; ++l)
            for (size_t k = ptr_[l]; k < end_[l]; ++k) regs_.push_back(lanes_[l][k].reg);
        std::sort(regs_.begin(), regs_.end());
        int visits = 0;   // most entries on one region
        for (size_t i = 0, j; i < regs_.size(); i = j) {
            for (j = i; j < regs_.size() && regs_[j] == regs_[i]; ++j) {}
            visits = std::max(visits, int(j - i));
        }
        regs_.erase(std::unique(regs_.begin(), regs_.end()), regs_.end());
        if (((int)regs_.size() > in_.cap || visits > kMaxSlotVisits) && maxn > 1) {
            split(0);
            split(1);
            return;
        }
        Window w;
        w.nslots = (int)regs_.size();
        w.entry_off = steps_ * kBatch;
        w.tab_off = (int64_t)tab_.size();
        for (int l = 0; l < kBatch; ++l) w.count[l] = int(end_[l] - ptr_[l]);
        w.nsteps = window_steps_of(w.count);
        tab_.insert(tab_.end(), regs_.begin(), regs_.end());
        windows_.push_back(w);
        steps_ += w.nsteps;
    }

    void range(double lo, double hi, bool last) {
        int maxn = 0;
        for (int l = 0; l < kBatch; ++l) {
            size_t e = ptr_[l];
            const auto &v = lanes_[l];
            while (e < v.size() && (last || v[e].s0 < hi)) ++e;
            end_[l] = e;
            maxn = std::max(maxn, int(e - ptr_[l]));
        }
        if (maxn == 0) return;
        regs_.clear();
        for (int l = 0; l < kBatch; ++l)
            for (size_t k = ptr_[l]; k < end_[l]; ++k) regs_.push_back(lanes_[l][k].reg);
        std::sort(regs_.begin(), regs_.end());
        regs_.erase(std::unique(regs_.begin(), regs_.end()), regs_.end());
        if ((int)regs_.size() > in_.cap && maxn > 1) {
            const double mid = 0.5 * (lo + hi);
            range(lo, mid, false);
            range(mid, hi, last);
            return;
        }
        Window w;
        w.nslots = (int)regs_.size();
        w.entry_off = steps_ * kBatch;
        w.tab_off = (int64_t)tab_.size();
        for (int l = 0; l < kBatch; ++l) w.count[l] = int(end_[l] - ptr_[l]);
        w.nsteps = window_steps_of(w.count);
        tab_.insert(tab_.end(), regs_.begin(), regs_.end());
        windows_.push_back(w);
        steps_ += w.nsteps;
        for (int l = 0; l < kBatch; ++l) ptr_[l] = end_[l];
    }

    const PackInput &in_;
    std::vector<std::vector<LaneSeg>> lanes_;
    std::vector<size_t> ptr_, end_;
    std::vector<int> regs_;
    std::vector<LaneSeg> tmp_;
    std::vector<Window> windows_;
    std::vector<int> tab_;
    int64_t steps_ = 0;
};

template <typename Seg>
void pack_impl(const PackInput &in, PackOutput &out, std::vector<Seg> &segs) {
    const int nb = (int)in.batch_first.size() - 1;
    if (in.cap < kBatch || in.cap > (1 << kSlotBits)) throw Error(MOC_EINVAL, "pack: slot cap out of range");
    if ((int64_t)in.mesh->R >= (int64_t(1) << (32 - kSlotBits)))
        throw Error(MOC_EINVAL, "pack: too many regions for the packed segment key");
    // pass 1: plan every batch, keep only the sizes
    std::vector<int64_t> b_steps(nb), b_win(nb), b_slots(nb), b_segs(nb), b_cross(nb);
    parallel_for(nb, in.n_threads, 4, [&](int64_t b0, int64_t b1, int) {
        BatchPlanner pl(in);
        for (int64_t b = b0; b < b1; ++b) {
            pl.plan(in.batch_first[b], in.batch_first[b + 1]);
            b_steps[b] = pl.steps();
            b_win[b] = pl.n_windows();
            b_slots[b] = pl.n_slots();
            b_segs[b] = pl.n_segments();
            b_cross[b] = pl.n_entries() - b_segs[b];
        }
    });
    std::vector<int64_t> e_off(nb + 1, 0), w_off(nb + 1, 0), s_off(nb + 1, 0);
    out.S = 0;
    out.crossings = 0;
    for (int b = 0; b < nb; ++b) {
        out.crossings += b_cross[b];
        e_off[b + 1] = e_off[b] + b_steps[b] * kBatch;
        w_off[b + 1] = w_off[b] + b_win[b];
        s_off[b + 1] = s_off[b] + b_slots[b];
        out.S += b_segs[b];
    }
    out.entries = e_off[nb];
    const int64_t nw = w_off[nb];
    out.batch_win.assign(w_off.begin(), w_off.end());
    out.win_entry_off.assign(nw, 0);
    out.win_nsteps.assign(nw, 0);
    out.win_tab_off.assign(nw, 0);
    out.win_nslots.assign(nw, 0);
    out.tab.assign(s_off[nb], 0);
    segs.assign((size_t)out.entries, Seg{});
    out.entry_region.assign(2 * (size_t)nb * kBatch, -1);
    std::vector<std::vector<double>> Vt(in.n_threads, std::vector<double>(in.mesh->R, 0.0));
    // pass 2: plan again (deterministic) and write
    parallel_for(nb, in.n_threads, 4, [&](int64_t b0, int64_t b1, int tid) {
        BatchPlanner pl(in);
        double *V = Vt[tid].data();
        for (int64_t b = b0; b < b1; ++b) {
            const int t0 = in.batch_first[b], t1 = in.batch_first[b + 1];
            pl.plan(t0, t1);
            if (pl.steps() != b_steps[b] || pl.n_slots() != b_slots[b])
                throw Error(MOC_EINVAL, "pack: non-deterministic batch plan");
            pl.write(segs.data() + e_off[b]);
            std::memcpy(out.tab.data() + s_off[b], pl.tab().data(), pl.tab().size() * sizeof(int));
            const auto &ws = pl.windows();
            for (size_t w = 0; w < ws.size(); ++w) {
                const int64_t i = w_off[b] + (int64_t)w;
                out.win_entry_off[i] = e_off[b] + ws[w].entry_off;
                out.win_nsteps[i] = ws[w].nsteps;
                out.win_tab_off[i] = s_off[b] + ws[w].tab_off;
                out.win_nslots[i] = ws[w].nslots;
            }
            const int R = in.mesh->R;
            for (int t = t0; t < t1; ++t) {
                const int l = t - t0;
                const auto &v = pl.lane(l);
                const int a = in.tracks->angle[t];
                const double wgt = in.quad->wa[a] * in.quad->delta[a];
                int first = -1, last = -1;
                for (const LaneSeg &s : v) {
                    if (s.reg >= R) continue;   // crossing entry
                    V[s.reg] += wgt * s.len;
                    if (first < 0) first = s.reg;
                    last = s.reg;
                }
                out.entry_region[(size_t)b * kBatch + l] = first;                       // sense 0
                out.entry_region[(size_t)nb * kBatch + (size_t)b * kBatch + l] = last;  // sense 1
            }
        }
    });
    out.V.assign(in.mesh->R, 0.0);
    for (const auto &vt : Vt)
        for (int r = 0; r < in.mesh->R; ++r) out.V[r] += vt[r];
}

}  // namespace

void find_coarse_surfaces(const Mesh &mesh, const Quadrature &quad, const Tracks &tracks,
                          const int *internal_of_user, int n_threads, CoarseSurfaces &cs) {
    struct CellSink : SegmentSink {
        const int *internal_of_user = nullptr;
        const CoarseSurfaces *cs = nullptr;
        std::vector<int64_t> *keys = nullptr;
        int prev = -1;
        void emit(int r, double) override {
            const int c = cs->cell_of[internal_of_user[r]];
            if (prev < 0) keys->push_back(cs->key(c, -1));
            else if (c != prev) keys->push_back(cs->key(std::min(c, prev), std::max(c, prev)));
            prev = c;
        }
    };
    const int nthr = std::max(1, n_threads);
    std::vector<std::vector<int64_t>> keys(nthr);
    parallel_for(tracks.T, nthr, 64, [&](int64_t t0, int64_t t1, int tid) {
        CellSink sink;
        sink.internal_of_user = internal_of_user;
        sink.cs = &cs;
        sink.keys = &keys[tid];
        for (int64_t t = t0; t < t1; ++t) {
            sink.prev = -1;
            trace_track(mesh, quad, tracks, (int)t, sink);
            if (sink.prev >= 0) keys[tid].push_back(cs.key(sink.prev, -1));
            auto &k = keys[tid];
            if (k.size() > (1u << 20)) {
                std::sort(k.begin(), k.end());
                k.erase(std::unique(k.begin(), k.end()), k.end());
            }
        }
    });
    std::vector<int64_t> all;
    for (auto &k : keys) all.insert(all.end(), k.begin(), k.end());
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    cs.a.resize(all.size());
    cs.b.resize(all.size());
    cs.id.clear();
    cs.id.reserve(all.size() * 2);
    for (size_t i = 0; i < all.size(); ++i) {
        cs.a[i] = int(all[i] / (cs.n_cells + 1)) - 1;
        cs.b[i] = int(all[i] % (cs.n_cells + 1)) - 1;
        cs.id[all[i]] = (int)i;
    }
}

void pack_segments_f32(const PackInput &in, PackOutput &out, std::vector<SegF> &segs) { pack_impl(in, out, segs); }
void pack_segments_f64(const PackInput &in, PackOutput &out, std::vector<SegD> &segs) { pack_impl(in, out, segs); }

}  // namespace moc
