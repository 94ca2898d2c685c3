// Test harness for the streaming server's scheduling core: a simulated
// device and clock behind the core's Executor interface, so the scheduling
// logic runs deterministically on the CPU.  The copy and compute queues are
// serial; each operation completes after a modelled duration.  Every copy,
// integrated frame and export is recorded, and the harness counts
// violations of what the core promises:
//   * a frame integrated twice;
//   * a host frame read from its ring slot before its copy completed, or a
//     ring slot overwritten while it holds a frame not yet integrated or
//     still being read;
//   * an export holding frames of another channel;
//   * more launches in flight than max_inflight;
//   * a channel attached to a slot another active channel holds, or
//     detached from a slot it does not hold.
// Its free device memory is a step in time (before, switch time, after),
// for admission by memory.
// Built by the tests with g++ together with csrc/xeng_sched.cpp.
#include <algorithm>
#include <cstdint>
#include <set>
#include <vector>

#include "xeng.h"
#include "xeng_sched.h"

using xeng::sched::Chan;
using xeng::sched::Job;

namespace {

struct SimTimes {
    double idle_us;      // clock advance when the core has nothing to do
    double copy_us;      // one frame's host-to-device copy
    double launch_us;    // fixed cost of a launch with work
    double frame_us;     // per integrated frame (all channels)
    double export_us;    // per export
};

class FakeExec : public xeng::sched::Executor {
public:
    FakeExec(const SimTimes &tm, int64_t ring_frames, int32_t max_inflight)
        : tm_(tm), ring_(ring_frames), max_inflight_(max_inflight) {}

    double now() override { return t; }

    void start() override {}   // the simulated clock runs on across runs

    int copy(const Chan &, int32_t chan, int64_t frame, int64_t *token) override
    {
        grow(chan);
        const double start = std::max(t, copy_free_);
        copy_free_ = start + tm_.copy_us * 1e-6;
        const size_t r = (size_t)(frame % ring_);
        RingSlot &rs = rings_[(size_t)chan][r];
        if (rs.pending || start < rs.busy_until) ++violations;   // overwrites a frame in use
        rs.frame = frame;
        rs.ready = copy_free_;
        rs.pending = true;
        copy_log.push_back(chan);
        copy_log.push_back(frame);
        *token = token_at(copy_free_, false);
        return XENG_OK;
    }

    int launch(const std::vector<Job> &jobs, const std::vector<Job> &exports, int64_t *token) override
    {
        int live = 0;
        for (size_t k = 0; k < done_at_.size(); ++k)
            if (is_launch_[k] && !released_[k]) ++live;
        if (live >= max_inflight_) ++violations;
        const double start = std::max(t, compute_free_);
        int64_t frames = 0;
        for (const Job &j : jobs) frames += j.f1 - j.f0;
        const double end = start + (jobs.empty() ? 0.0 : tm_.launch_us * 1e-6) + frames * tm_.frame_us * 1e-6 +
                           (double)exports.size() * tm_.export_us * 1e-6;
        for (const Job &j : jobs) {
            grow(j.chan);
            for (int64_t f = j.f0; f < j.f1; ++f) {
                if (host_[(size_t)j.chan]) {
                    RingSlot &rs = rings_[(size_t)j.chan][(size_t)(f % ring_)];
                    if (rs.frame != f || rs.ready > start) ++violations;   // stale or unfinished copy
                    rs.pending = false;
                    rs.busy_until = std::max(rs.busy_until, end);
                }
                if (!integrated_[(size_t)j.chan].insert(f).second) ++violations;   // twice
                acc_[(size_t)j.slot].push_back({j.chan, f});
                int_log.push_back(launches);
                int_log.push_back(j.chan);
                int_log.push_back(f);
            }
        }
        for (const Job &e : exports) {
            std::vector<std::pair<int32_t, int64_t>> &a = acc_[(size_t)e.slot];
            exp_log.push_back(e.chan);
            exp_log.push_back(e.slot);
            exp_log.push_back(e.f0);
            exp_log.push_back(e.f1);
            exp_log.push_back((int64_t)exp_frames.size());
            exp_log.push_back((int64_t)a.size());
            for (const auto &p : a) {
                if (p.first != e.chan) ++violations;   // another channel's frames
                exp_frames.push_back(p.second);
            }
            a.clear();
        }
        compute_free_ = end;
        if (!jobs.empty()) ++launches;
        *token = token_at(end, true);
        return XENG_OK;
    }

    int64_t free_bytes() override { return t < free_switch_ ? free_before_ : free_after_; }

    int attach(const Chan &, int32_t chan, int32_t slot, bool new_slot, bool new_ring) override
    {
        grow(chan);
        if (holder_[(size_t)slot] >= 0) ++violations;
        holder_[(size_t)slot] = chan;
        attach_log.push_back(chan);
        attach_log.push_back(slot);
        attach_log.push_back(new_slot ? 1 : 0);
        attach_log.push_back(new_ring ? 1 : 0);
        attach_log.push_back((int64_t)(t * 1e9));
        return XENG_OK;
    }

    int detach(const Chan &, int32_t chan, int32_t slot) override
    {
        if (holder_[(size_t)slot] != chan) ++violations;
        holder_[(size_t)slot] = -1;
        acc_[(size_t)slot].clear();
        ++resets;
        return XENG_OK;
    }

    void set_free(int64_t before, double t_switch, int64_t after)
    {
        free_before_ = before;
        free_switch_ = t_switch;
        free_after_ = after;
    }

    int poll(int64_t token, bool wait) override
    {
        const double d = done_at_[(size_t)token];
        if (wait && d > t) t = d;
        return d <= t ? 1 : 0;
    }

    void release(int64_t token) override { released_[(size_t)token] = true; }

    void idle() override { t += tm_.idle_us * 1e-6; }

    void set_slots(int32_t slots)
    {
        acc_.resize((size_t)slots);
        holder_.assign((size_t)slots, -1);
    }
    void set_host(int32_t chan, bool host)
    {
        grow(chan);
        host_[(size_t)chan] = host;
    }

    double t = 0;
    int64_t violations = 0, launches = 0, resets = 0;
    std::vector<int64_t> copy_log, int_log, exp_log, exp_frames, attach_log;

private:
    struct RingSlot {
        int64_t frame = -1;
        double ready = 0;       // its copy's completion
        double busy_until = 0;  // completion of the last launch reading it
        bool pending = false;   // copied, not yet handed to a launch
    };

    void grow(int32_t chan)
    {
        while ((int32_t)rings_.size() <= chan) {
            rings_.emplace_back((size_t)ring_);
            integrated_.emplace_back();
            host_.push_back(false);
        }
    }

    int64_t token_at(double when, bool launch)
    {
        done_at_.push_back(when);
        is_launch_.push_back(launch);
        released_.push_back(false);
        return (int64_t)done_at_.size() - 1;
    }

    SimTimes tm_;
    int64_t ring_;
    int32_t max_inflight_;
    double copy_free_ = 0, compute_free_ = 0;
    std::vector<double> done_at_;
    std::vector<bool> is_launch_, released_;
    std::vector<std::vector<RingSlot>> rings_;
    std::vector<std::set<int64_t>> integrated_;
    std::vector<bool> host_;
    std::vector<std::vector<std::pair<int32_t, int64_t>>> acc_;   // per slot: (channel, frame) since export
    std::vector<int32_t> holder_;   // per slot: the attached channel, -1 if none
    int64_t free_before_ = INT64_C(1) << 50, free_after_ = INT64_C(1) << 50;
    double free_switch_ = 0;
};

struct Sim {
    xeng::sched::Scheduler sch;
    FakeExec ex;
    Sim(const xeng::sched::Config &c, const SimTimes &tm) : sch(c), ex(tm, c.ring_frames, c.max_inflight)
    {
        ex.set_slots(c.slots);
    }
};

const std::vector<int64_t> *log_of(const Sim *s, int which)
{
    switch (which) {
    case 0: return &s->ex.copy_log;
    case 1: return &s->ex.int_log;
    case 2: return &s->ex.exp_log;
    case 3: return &s->ex.exp_frames;
    case 4: return &s->ex.attach_log;
    default: return nullptr;
    }
}

}  // namespace

extern "C" {

// cfg: frame_len, dump_frames, ring_frames, max_inflight, slots, stagger,
// slot_bytes, ring_bytes, mem_budget, mem_reserve; per: frame_period_us,
// launch_period_us; tm: idle, copy, launch, frame, export (us).
void *sim_create(const int64_t *cfg, const double *per, const double *tm)
{
    xeng::sched::Config c;
    c.frame_len = cfg[0];
    c.dump_frames = cfg[1];
    c.ring_frames = cfg[2];
    c.max_inflight = (int32_t)cfg[3];
    c.slots = (int32_t)cfg[4];
    c.stagger_exports = cfg[5] != 0;
    c.slot_bytes = cfg[6];
    c.ring_bytes = cfg[7];
    c.mem_budget = cfg[8];
    c.mem_reserve = cfg[9];
    c.frame_period_us = per[0];
    c.launch_period_us = per[1];
    c.pairs = 1.0;
    return new Sim(c, SimTimes{tm[0], tm[1], tm[2], tm[3], tm[4]});
}

void sim_destroy(void *h) { delete static_cast<Sim *>(h); }

void sim_set_free(void *h, int64_t before, double t_switch, int64_t after)
{
    static_cast<Sim *>(h)->ex.set_free(before, t_switch, after);
}

int32_t sim_admit(void *h, int64_t src_frames, int32_t host, double start_s, int64_t total_frames)
{
    Sim *s = static_cast<Sim *>(h);
    const int32_t k = s->sch.admit(src_frames, host != 0, start_s, total_frames);
    s->ex.set_host(k, host != 0);
    return k;
}

// stats: released, done, dropped, launches, dumps, backlog, violations,
// resets, waiting, device_bytes (int64); seconds, p50_ms, p99_ms, max_ms
// (double)
int sim_run(void *h, double seconds, int64_t *istats, double *dstats)
{
    Sim *s = static_cast<Sim *>(h);
    xeng::sched::Stats st;
    const int rc = s->sch.run(s->ex, seconds, &st);
    istats[0] = st.frames_released;
    istats[1] = st.frames_done;
    istats[2] = st.frames_dropped;
    istats[3] = st.launches;
    istats[4] = st.dumps;
    istats[5] = st.backlog_frames;
    istats[6] = s->ex.violations;
    istats[7] = s->ex.resets;
    istats[8] = st.waiting;
    istats[9] = st.device_bytes;
    dstats[0] = st.seconds;
    dstats[1] = st.p50_ms;
    dstats[2] = st.p99_ms;
    dstats[3] = st.max_ms;
    return rc;
}

int64_t sim_log_size(void *h, int which)
{
    const std::vector<int64_t> *v = log_of(static_cast<Sim *>(h), which);
    return v ? (int64_t)v->size() : -1;
}

void sim_log_copy(void *h, int which, int64_t *dst)
{
    const std::vector<int64_t> *v = log_of(static_cast<Sim *>(h), which);
    if (v) std::copy(v->begin(), v->end(), dst);
}

// state, slot, released, done, dumps, last_dump_first, start_s * 1e9,
// admitted_s * 1e9 (-1: never)
void sim_chan(void *h, int32_t k, int64_t *out)
{
    const Chan &c = static_cast<Sim *>(h)->sch.chans()[(size_t)k];
    out[0] = c.state;
    out[1] = c.slot;
    out[2] = c.released;
    out[3] = c.done;
    out[4] = c.dumps;
    out[5] = c.last_dump_first;
    out[6] = (int64_t)(c.start_s * 1e9);
    out[7] = c.admitted_s < 0 ? -1 : (int64_t)(c.admitted_s * 1e9);
}

}  // extern "C"
