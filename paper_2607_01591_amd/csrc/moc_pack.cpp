// Device packing of the traced segments into sweep batches and tally windows.
//
// A batch is up to 64 adjacent parallel tracks of one angle (one per lane of a
// wavefront). Each batch is cut along the track direction into windows of about
// `window_len` cm: lane l's part of window w holds its segments whose start lies in
// [w L, (w + 1) L). Within a window the lanes advance in lockstep (shorter lanes are
// padded with zero-length steps), and every distinct region the window touches gets a
// window-local tally slot, so the sweep kernel can accumulate the window's tallies in
// LDS and flush each slot once. A window whose slot count exceeds `cap` is split in half
// by distance.
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
    int reg;      // internal region
    double len;
    double s0;    // distance of the segment start from the track start (sense 0)
};

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
                for (int j = 0; j < w.nsteps; ++j) {
                    Seg &e = segs[w.entry_off + (int64_t)j * kBatch + l];
                    if (j < w.count[l]) {
                        const LaneSeg &s = v[p[l] + j];
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
        regs_.erase(std::unique(regs_.begin(), regs_.end()), regs_.end());
        if ((int)regs_.size() > in_.cap && maxn > 1) {
            split(0);
            split(1);
            return;
        }
        Window w;
        w.nsteps = maxn;
        w.nslots = (int)regs_.size();
        w.entry_off = steps_ * kBatch;
        w.tab_off = (int64_t)tab_.size();
        for (int l = 0; l < kBatch; ++l) w.count[l] = int(end_[l] - ptr_[l]);
        tab_.insert(tab_.end(), regs_.begin(), regs_.end());
        windows_.push_back(w);
        steps_ += maxn;
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
        w.nsteps = maxn;
        w.nslots = (int)regs_.size();
        w.entry_off = steps_ * kBatch;
        w.tab_off = (int64_t)tab_.size();
        for (int l = 0; l < kBatch; ++l) w.count[l] = int(end_[l] - ptr_[l]);
        tab_.insert(tab_.end(), regs_.begin(), regs_.end());
        windows_.push_back(w);
        steps_ += maxn;
        for (int l = 0; l < kBatch; ++l) ptr_[l] = end_[l];
    }

    const PackInput &in_;
    std::vector<std::vector<LaneSeg>> lanes_;
    std::vector<size_t> ptr_, end_;
    std::vector<int> regs_;
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
    std::vector<int64_t> b_steps(nb), b_win(nb), b_slots(nb), b_segs(nb);
    parallel_for(nb, in.n_threads, 4, [&](int64_t b0, int64_t b1, int) {
        BatchPlanner pl(in);
        for (int64_t b = b0; b < b1; ++b) {
            pl.plan(in.batch_first[b], in.batch_first[b + 1]);
            b_steps[b] = pl.steps();
            b_win[b] = pl.n_windows();
            b_slots[b] = pl.n_slots();
            b_segs[b] = pl.n_segments();
        }
    });
    std::vector<int64_t> e_off(nb + 1, 0), w_off(nb + 1, 0), s_off(nb + 1, 0);
    out.S = 0;
    for (int b = 0; b < nb; ++b) {
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
            for (int t = t0; t < t1; ++t) {
                const int l = t - t0;
                const auto &v = pl.lane(l);
                const int a = in.tracks->angle[t];
                const double wgt = in.quad->wa[a] * in.quad->delta[a];
                for (const LaneSeg &s : v) V[s.reg] += wgt * s.len;
                if (!v.empty()) {
                    out.entry_region[(size_t)b * kBatch + l] = v.front().reg;                       // sense 0
                    out.entry_region[(size_t)nb * kBatch + (size_t)b * kBatch + l] = v.back().reg;  // sense 1
                }
            }
        }
    });
    out.V.assign(in.mesh->R, 0.0);
    for (const auto &vt : Vt)
        for (int r = 0; r < in.mesh->R; ++r) out.V[r] += vt[r];
}

}  // namespace

void pack_segments_f32(const PackInput &in, PackOutput &out, std::vector<SegF> &segs) { pack_impl(in, out, segs); }
void pack_segments_f64(const PackInput &in, PackOutput &out, std::vector<SegD> &segs) { pack_impl(in, out, segs); }

}  // namespace moc
