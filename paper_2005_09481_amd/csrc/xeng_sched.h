// Scheduling core of the streaming server (Sec. 2.1: every channel delivers
// a sample every 2.56 us, integrated on the device and exported at a
// cadence).  It decides, in real time:
//   * releases: frame f of a channel becomes due at start + f * frame_period;
//     a host-sourced frame is first copied into the channel's device ring of
//     ring_frames frames, and is dropped (recorded as a gap, never
//     integrated) while that ring still holds frames not yet integrated;
//   * continuous batching: about every launch_period, one launch takes every
//     channel's available frames up to its next export boundary, a ring wrap
//     or a gap, while up to max_inflight earlier launches may still run;
//   * exports: a channel whose launched frames reach an export boundary is
//     exported (with reset) right after that launch; boundaries every
//     dump_frames frames, offset by slot * dump_frames / slots when exports
//     are staggered;
//   * admission by memory: waiting channels, in order of arrival, take a
//     free slot once the device memory they need is there -- the slot's
//     accumulators and export buffer at its first use, a ring for a host
//     source unless a finished channel left one -- within the server's
//     budget and within the device's free memory at that moment (less a
//     reserve); a slot's memory and a finished channel's ring stay with the
//     server for the next channel;
//   * latency of a frame: from its release time to the completion of the
//     launch that integrated it.
// It makes no device call.  An Executor carries out copies, launches,
// exports and resets and reports their completion and the time, so the same
// logic drives the HIP server and a simulated device with a simulated clock.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <utility>
#include <vector>

namespace xeng {
namespace sched {

struct Config {
    int64_t frame_len = 0;      // samples per frame
    int64_t dump_frames = 0;    // frames per export
    int64_t ring_frames = 0;    // frames in a host source's device ring
    int32_t max_inflight = 1;   // launches queued at once
    int32_t slots = 0;          // channels integrating at once
    double frame_period_us = 0;
    double launch_period_us = 0;
    bool stagger_exports = false;
    double pairs = 0;           // N(N+1)/2, for the CMAC rate
    int64_t slot_bytes = 0;     // device bytes a slot takes at its first use
    int64_t ring_bytes = 0;     // device bytes of a host source's ring
    int64_t mem_budget = 0;     // most device bytes the server may hold (0: no budget)
    int64_t mem_reserve = 0;    // device bytes admission leaves free
};

struct Chan {
    int state = 0;                 // 0 waiting for a slot, 1 active, 2 finished
    int32_t slot = -1;
    double admitted_s = -1;        // when it took its slot (seconds into the run)
    bool host = false;             // frames copied from host memory into a device ring
    int64_t src_frames = 0;        // distinct source frames, cycled
    double start_s = 0;            // release time of frame 0 (seconds into the run)
    int64_t total_frames = 0;      // 0: unlimited
    int64_t released = 0;          // frames whose release time has passed
    int64_t available = 0;         // frames the device may read (copied, for a host source)
    int64_t launched = 0;          // frames handed to launches (or passed over as dropped)
    int64_t done = 0;              // frames whose launch has completed
    int64_t dumps = 0;
    int64_t last_dump_first = -1;  // first frame of the last exported integration
    int64_t phase = 0;             // exports at frame counts m * dump_frames - phase
    std::deque<std::pair<int64_t, int64_t>> copies;   // (frames copied up to, completion token)
    std::deque<int64_t> gaps;      // frames dropped at ingest, in order
};

// Frames [f0, f1) of channel `chan` (slot `slot`).  As an export: the
// channel's integration that ends at frame f1 (= its export boundary).
struct Job {
    int32_t chan;
    int32_t slot;
    int64_t f0, f1;
};

struct Stats {
    int64_t frames_released = 0, frames_done = 0, frames_dropped = 0;
    int64_t launches = 0, dumps = 0, backlog_frames = 0;
    int64_t waiting = 0;           // channels still waiting for a slot or memory at the end
    int64_t device_bytes = 0;      // device memory the server holds for slots and rings
    double seconds = 0, tcmacs = 0, p50_ms = 0, p99_ms = 0, max_ms = 0;
    // where the real-time loop's time went: its longest pass, and the
    // longest single launch (with its exports) and ingest copy it queued
    double max_pass_ms = 0, max_launch_call_ms = 0, max_copy_call_ms = 0;
};

// Status values are the library's (0 = ok, < 0 = error).
class Executor {
public:
    virtual ~Executor() = default;
    // seconds since the run began (since start())
    virtual double now() = 0;
    // the run's clock starts: called once per run, after the channels that
    // could be admitted before it were (their allocations stall no stream)
    virtual void start() = 0;
    // host source: start copying frame `frame` of channel `chan` into its
    // ring slot frame % ring_frames; `token` names the copy's completion
    // (an executor may hold copies back until flush)
    virtual int copy(const Chan &c, int32_t chan, int64_t frame, int64_t *token) = 0;
    // start every copy held back so far: called once per pass of the loop,
    // after its releases
    virtual int flush() { return 0; }
    // one batched launch over `jobs` (possibly none), then the exports, in
    // order after everything queued before; `token` names its completion
    virtual int launch(const std::vector<Job> &jobs, const std::vector<Job> &exports, int64_t *token) = 0;
    // device bytes free right now
    virtual int64_t free_bytes() = 0;
    // channel `chan` enters `slot`: allocate the slot's memory if `new_slot`
    // and one more ring if `new_ring`, and give a host source a ring.
    // XENG_ENOMEM, with nothing allocated, leaves the channel waiting.
    virtual int attach(const Chan &c, int32_t chan, int32_t slot, bool new_slot, bool new_ring) = 0;
    // channel `chan` finished: zero its slot, in order after everything
    // queued before, and keep its ring (if any) for the next host source
    virtual int detach(const Chan &c, int32_t chan, int32_t slot) = 0;
    // 1 complete, 0 not yet; `wait` blocks until complete
    virtual int poll(int64_t token, bool wait) = 0;
    // the token will not be polled again
    virtual void release(int64_t token) = 0;
    // nothing to do right now
    virtual void idle() = 0;
};

class Scheduler {
public:
    explicit Scheduler(const Config &cfg);
    // a new channel; it waits for admission (at the start of the next run,
    // or later if no slot or memory is free)
    int32_t admit(int64_t src_frames, bool host, double start_s, int64_t total_frames);
    // the real-time loop for `seconds`, then wait for what is queued
    int run(Executor &ex, double seconds, Stats *stats);

    const Config &config() const { return cfg_; }
    const std::vector<Chan> &chans() const { return chans_; }
    int32_t slot_owner(int32_t slot) const { return slot_owner_[(std::size_t)slot]; }

private:
    double release_time(const Chan &c, int64_t f) const { return c.start_s + (double)f * cfg_.frame_period_us * 1e-6; }
    int64_t export_phase(int32_t slot) const;
    int admit_waiting(Executor &ex, double t, bool before_start, bool *admitted);
    int64_t bytes_held() const { return slots_with_mem_ * cfg_.slot_bytes + rings_held_ * cfg_.ring_bytes; }

    Config cfg_;
    std::vector<Chan> chans_;
    std::vector<int32_t> free_slots_;
    std::vector<int32_t> slot_owner_;   // channel using each slot, -1 if none
    std::vector<char> slot_mem_;        // slots whose memory exists
    int64_t slots_with_mem_ = 0;
    int64_t rings_held_ = 0;            // rings allocated
    int64_t rings_free_ = 0;            // rings left by finished channels
    size_t next_waiting_ = 0;           // no channel before it waits
};

}  // namespace sched
}  // namespace xeng
