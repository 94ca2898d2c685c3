// Scheduling core of the streaming server; see xeng_sched.h.  No device
// calls: everything that touches the device goes through the Executor.
#include "xeng_sched.h"

#include <algorithm>
#include <climits>

#include "../../include/xeng.h"

namespace xeng {
namespace sched {

namespace {

struct Range {
    int32_t chan;
    int64_t f0, f1;   // frames [f0, f1)
    bool skipped;     // dropped frames passed over: neither integrated nor counted as done work
};

struct InFlight {
    int64_t token = -1;
    std::vector<Range> ranges;
};

}  // namespace

Scheduler::Scheduler(const Config &cfg) : cfg_(cfg)
{
    for (int32_t k = cfg_.slots - 1; k >= 0; --k) free_slots_.push_back(k);
    slot_owner_.assign((size_t)cfg_.slots, -1);
    slot_mem_.assign((size_t)cfg_.slots, 0);
}

int64_t Scheduler::export_phase(int32_t slot) const
{
    if (!cfg_.stagger_exports) return 0;
    return (int64_t)slot * cfg_.dump_frames / (int64_t)cfg_.slots;
}

int32_t Scheduler::admit(int64_t src_frames, bool host, double start_s, int64_t total_frames)
{
    Chan c;
    c.host = host;
    c.src_frames = src_frames;
    c.start_s = start_s;
    c.total_frames = total_frames;
    chans_.push_back(c);
    return (int32_t)chans_.size() - 1;
}

// Admits at most one waiting channel (in the loop, an admission may
// allocate, and the channels already streaming are served between
// admissions).  Before the run's clock starts, the admission time is set
// once it has started.
int Scheduler::admit_waiting(Executor &ex, double t, bool before_start, bool *admitted_out)
{
    bool admitted = false;
    *admitted_out = false;
    for (; next_waiting_ < chans_.size() && !admitted; ++next_waiting_) {
        Chan &c = chans_[next_waiting_];
        if (c.state != 0) continue;
        if (free_slots_.empty()) return XENG_OK;
        // a free slot whose memory exists, else the most recently freed one
        size_t pick = free_slots_.size() - 1;
        for (size_t k = free_slots_.size(); k-- > 0;)
            if (slot_mem_[(size_t)free_slots_[k]]) {
                pick = k;
                break;
            }
        const int32_t slot = free_slots_[pick];
        const bool new_slot = !slot_mem_[(size_t)slot];
        const bool new_ring = c.host && rings_free_ == 0;
        const int64_t need = (new_slot ? cfg_.slot_bytes : 0) + (new_ring ? cfg_.ring_bytes : 0);
        if (need > 0) {
            if (cfg_.mem_budget > 0 && bytes_held() + need > cfg_.mem_budget) return XENG_OK;
            if (need > ex.free_bytes() - cfg_.mem_reserve) return XENG_OK;
        }
        const int rc = ex.attach(c, (int32_t)next_waiting_, slot, new_slot, new_ring);
        if (rc == XENG_ENOMEM) return XENG_OK;   // the device had less than it said: wait
        if (rc != XENG_OK) return rc;
        if (new_slot) {
            slot_mem_[(size_t)slot] = 1;
            ++slots_with_mem_;
        }
        if (new_ring) {
            ++rings_held_;
            ++rings_free_;
        }
        if (c.host) --rings_free_;
        free_slots_.erase(free_slots_.begin() + (std::ptrdiff_t)pick);
        c.slot = slot;
        c.state = 1;
        c.phase = export_phase(slot);
        // its stream starts once admitted (and its memory is ready: taken
        // after attach, which may have allocated)
        if (!before_start) {
            const double ta = std::max(t, ex.now());
            c.admitted_s = ta;
            if (c.start_s < ta) c.start_s = ta;
        }
        slot_owner_[(size_t)slot] = (int32_t)next_waiting_;
        admitted = true;
        *admitted_out = true;
    }
    return XENG_OK;
}

int Scheduler::run(Executor &ex, double seconds, Stats *stats)
{
    const Config &cf = cfg_;
    std::vector<float> lat;
    std::deque<InFlight> inflight;
    int64_t dropped = 0, launches = 0, frames_done = 0;
    double next_launch = 0;
    int rc = XENG_OK;

    auto retire = [&](bool wait) -> int {
        while (!inflight.empty()) {
            InFlight &f = inflight.front();
            const int q = ex.poll(f.token, wait);
            if (q < 0) return q;
            if (q == 0) return XENG_OK;
            const double t = ex.now();
            for (const Range &r : f.ranges) {
                Chan &c = chans_[(size_t)r.chan];
                if (!r.skipped) {
                    for (int64_t fr = r.f0; fr < r.f1; ++fr)
                        lat.push_back((float)(1e3 * (t - release_time(c, fr))));
                    frames_done += r.f1 - r.f0;
                }
                c.done = r.f1;
                if (c.state == 1 && c.total_frames > 0 && c.done >= c.total_frames) {
                    // finished: zero what it integrated past its last export
                    // (queued behind that export), free the slot and keep
                    // the ring
                    c.state = 2;
                    const int e = ex.detach(c, r.chan, c.slot);
                    if (e != XENG_OK) return e;
                    free_slots_.push_back(c.slot);
                    if (c.host) ++rings_free_;
                }
            }
            ex.release(f.token);
            inflight.pop_front();
        }
        return XENG_OK;
    };

    // every channel that fits now is admitted before the clock starts
    for (bool more = true; more && rc == XENG_OK;) rc = admit_waiting(ex, 0.0, true, &more);
    ex.start();
    const double t_start = ex.now();
    for (Chan &c : chans_)
        if (c.state == 1 && c.admitted_s < 0) {
            c.admitted_s = t_start;
            if (c.start_s < t_start) c.start_s = t_start;
        }

    double prev_pass = -1, max_pass = 0, max_launch_call = 0, max_copy_call = 0;
    while (rc == XENG_OK) {
        const double t = ex.now();
        if (prev_pass >= 0) max_pass = std::max(max_pass, t - prev_pass);
        prev_pass = t;
        if (t >= seconds) break;
        // admissions into free slots, by memory
        bool admitted = false;
        if ((rc = admit_waiting(ex, t, false, &admitted)) != XENG_OK) break;
        // releases (and ingest copies for host sources)
        for (size_t k = 0; k < chans_.size() && rc == XENG_OK; ++k) {
            Chan &c = chans_[k];
            if (c.state != 1) continue;
            const int64_t limit = c.total_frames > 0 ? c.total_frames : INT64_MAX;
            while (c.released < limit && release_time(c, c.released) <= t) {
                const int64_t f = c.released++;
                if (!c.host) {
                    c.available = c.released;
                    continue;
                }
                if (f - c.done >= cf.ring_frames) {
                    // the ring still holds frames not yet integrated: lost,
                    // and passed over by the launches
                    ++dropped;
                    c.gaps.push_back(f);
                    continue;
                }
                int64_t tok = -1;
                const double tc = ex.now();
                if ((rc = ex.copy(c, (int32_t)k, f, &tok)) != XENG_OK) break;
                max_copy_call = std::max(max_copy_call, ex.now() - tc);
                c.copies.push_back({f + 1, tok});
            }
            while (rc == XENG_OK && !c.copies.empty()) {
                const int q = ex.poll(c.copies.front().second, false);
                if (q < 0) rc = q;
                if (q <= 0) break;
                c.available = c.copies.front().first;
                ex.release(c.copies.front().second);
                c.copies.pop_front();
            }
        }
        if (rc != XENG_OK) break;
        // the pass's ingest copies, together
        {
            const double tc = ex.now();
            if ((rc = ex.flush()) != XENG_OK) break;
            max_copy_call = std::max(max_copy_call, ex.now() - tc);
        }
        if ((rc = retire(false)) != XENG_OK) break;
        // one batched launch over every channel's available frames
        if (t >= next_launch && (int)inflight.size() < cf.max_inflight) {
            std::vector<Job> jobs, exports;
            InFlight f;
            for (size_t k = 0; k < chans_.size(); ++k) {
                Chan &c = chans_[k];
                if (c.state != 1) continue;
                int64_t f0 = c.launched;
                const int64_t boundary = ((f0 + c.phase) / cf.dump_frames + 1) * cf.dump_frames - c.phase;
                // pass over dropped frames at the front, up to the export boundary
                int64_t g = f0;
                while (!c.gaps.empty() && c.gaps.front() == g && g < boundary) {
                    c.gaps.pop_front();
                    ++g;
                }
                if (g > f0) {
                    f.ranges.push_back({(int32_t)k, f0, g, true});
                    c.launched = f0 = g;
                    if (g == boundary) {
                        exports.push_back({(int32_t)k, c.slot, std::max<int64_t>(0, g - cf.dump_frames), g});
                        continue;
                    }
                }
                if (c.available <= f0) continue;
                const int64_t wrap_n = c.host ? cf.ring_frames : c.src_frames;
                const int64_t wrap = (f0 / wrap_n + 1) * wrap_n;
                const int64_t next_gap = c.gaps.empty() ? INT64_MAX : c.gaps.front();
                const int64_t f1 = std::min({c.available, boundary, wrap, next_gap});
                jobs.push_back({(int32_t)k, c.slot, f0, f1});
                f.ranges.push_back({(int32_t)k, f0, f1, false});
                c.launched = f1;
                if (f1 == boundary) exports.push_back({(int32_t)k, c.slot, std::max<int64_t>(0, f1 - cf.dump_frames), f1});
            }
            if (!f.ranges.empty()) {
                const double tl = ex.now();
                if ((rc = ex.launch(jobs, exports, &f.token)) != XENG_OK) break;
                max_launch_call = std::max(max_launch_call, ex.now() - tl);
                for (const Job &e : exports) {
                    Chan &c = chans_[(size_t)e.chan];
                    c.last_dump_first = e.f0;
                    ++c.dumps;
                }
                inflight.push_back(std::move(f));
                if (!jobs.empty()) ++launches;
                next_launch = t + cf.launch_period_us * 1e-6;
            }
        }
        ex.idle();
    }
    const int rc2 = retire(true);
    if (rc == XENG_OK) rc = rc2;
    const double wall = ex.now();
    *stats = Stats();
    int64_t released = 0;
    for (const Chan &c : chans_) {
        released += c.released;
        stats->dumps += c.dumps;
    }
    stats->frames_released = released;
    stats->frames_done = frames_done;
    stats->frames_dropped = dropped;
    stats->launches = launches;
    stats->seconds = wall;
    stats->tcmacs = wall > 0 ? (double)frames_done * (double)cf.frame_len * cf.pairs / wall / 1e12 : 0.0;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) { return (double)lat[std::min(lat.size() - 1, (size_t)(p * (double)lat.size()))]; };
        stats->p50_ms = pct(0.50);
        stats->p99_ms = pct(0.99);
        stats->max_ms = lat.back();
    }
    stats->backlog_frames = released - frames_done - dropped;
    for (const Chan &c : chans_) stats->waiting += c.state == 0 ? 1 : 0;
    stats->device_bytes = bytes_held();
    stats->max_pass_ms = 1e3 * max_pass;
    stats->max_launch_call_ms = 1e3 * max_launch_call;
    stats->max_copy_call_ms = 1e3 * max_copy_call;
    return rc;
}

}  // namespace sched
}  // namespace xeng
