// Streaming correlation server: channels ingest frames at the instrument's
// sample rate, the device accumulators integrate them, and every channel
// exports its visibilities each `dump_frames` frames (Sec. 2.1: samples every
// 2.56 us per channel; integrated visibilities exported at a cadence).
//
// One call, xeng_server_run, drives a real-time loop on the calling thread:
//   * releases: frame f of a channel becomes available at its release time
//     start + stagger + f * frame_period (for a host source, once its copy
//     into the channel's device ring has completed);
//   * continuous batching: about every launch_period, one batched launch
//     correlates every channel's available frames (up to its next dump
//     boundary), while earlier launches may still run on the device;
//   * exports: a channel reaching a dump boundary is dumped (with reset)
//     into its own device buffer right after the launch that completed it
//     (boundaries every dump_frames frames, offset per slot with
//     XENG_SERVER_STAGGER_EXPORTS);
//   * admission: a channel admitted while every slot is in use waits and
//     takes the first slot released by a channel that has finished;
//   * latency of a frame: from its release time to the host observing the
//     completion of the launch that integrated it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "../../include/xeng.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Chan {
    int state = 0;                 // 0 waiting for a slot, 1 active, 2 finished
    int32_t slot = -1;
    const uint8_t *src = nullptr;  // [src_frames][frame_len][N]
    int src_host = 0;
    int64_t src_frames = 0;
    double start_s = 0;            // release time of frame 0 (seconds after run start)
    int64_t total_frames = 0;      // 0: unlimited
    int64_t released = 0;          // frames whose release time has passed
    int64_t available = 0;         // frames the device may read (copied, for a host source)
    int64_t launched = 0;          // frames handed to launches
    int64_t done = 0;              // frames whose launch has completed
    int64_t dumps = 0;
    int64_t last_dump_first = -1;  // first frame of the last exported integration
    int64_t phase = 0;             // exports at frame counts m * dump_frames - phase
    uint8_t *ring = nullptr;       // device ring for a host source
    std::deque<std::pair<int64_t, hipEvent_t>> copies;   // (frames copied up to, event)
    std::deque<int64_t> gaps;      // frames dropped at ingest, in order: never integrated
};

struct Range {
    int32_t chan;
    int64_t f0, f1;     // frames [f0, f1)
    bool skipped;       // dropped frames passed over: neither integrated nor counted as done work
};

struct InFlight {
    hipEvent_t ev = nullptr;
    std::vector<Range> ranges;
};

}  // namespace

struct xeng_server {
    xeng_server_config cfg;
    xeng_ctx *ctx = nullptr;
    int32_t *d_out = nullptr;            // max_channels dump buffers
    int64_t out_i32 = 0;                 // per buffer
    int64_t frame_bytes = 0;
    std::vector<Chan> chans;
    std::vector<int32_t> free_slots;
    std::vector<int32_t> slot_owner;     // channel using each slot, -1 if none
    hipStream_t compute = nullptr, copy = nullptr;
    std::vector<hipEvent_t> event_pool;
};

namespace {

hipEvent_t get_event(xeng_server *s)
{
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Export phase of a slot (XENG_SERVER_STAGGER_EXPORTS), else 0.
int64_t export_phase(const xeng_server *s, int32_t slot)
{
    if (!(s->cfg.flags & XENG_SERVER_STAGGER_EXPORTS)) return 0;
    return (int64_t)slot * s->cfg.dump_frames / (int64_t)s->slot_owner.size();
}

double release_time(const xeng_server *s, const Chan &c, int64_t f)
{
    return c.start_s + (double)f * s->cfg.frame_period_us * 1e-6;
}

void destroy_server(xeng_server *s)
{
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (Chan &c : s->chans) {
        for (auto &cp : c.copies) s->event_pool.push_back(cp.second);
        if (c.ring) (void)hipFree(c.ring);
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->ctx) (void)xeng_destroy(s->ctx);
    delete s;
}

}  // namespace

extern "C" {

int xeng_server_create(const xeng_server_config *cfg, xeng_server **out)
{
    if (!cfg || !out) return XENG_EINVAL;
    *out = nullptr;
    if (cfg->n_inputs < 1 || cfg->n_inputs > 65535 || cfg->frame_len < 1 || cfg->dump_frames < 1 ||
        cfg->ring_frames < 1 || cfg->frame_period_us <= 0 || cfg->launch_period_us < 0 || cfg->max_inflight < 1 ||
        cfg->max_channels < 0 || cfg->mem_budget_bytes < 0 || cfg->reserved != 0 ||
        (cfg->flags & ~(XENG_NIBBLE_RE_LOW | XENG_SERVER_STAGGER_EXPORTS)) ||
        (int64_t)cfg->frame_len * cfg->dump_frames > xeng_max_integration())
        return XENG_EINVAL;
    const int64_t n = cfg->n_inputs;
    const int64_t frame_bytes = (int64_t)cfg->frame_len * n;
    const int64_t out_bytes = n * (n + 1) / 2 * 8;
    // device bytes per channel: accumulators, export buffer and (for host
    // sources) the ingest ring
    const int64_t per_chan = xeng_slot_bytes(cfg->n_inputs) + out_bytes + (int64_t)cfg->ring_frames * frame_bytes;
    int64_t chans = cfg->max_channels;
    if (cfg->mem_budget_bytes > 0) chans = std::min<int64_t>(chans > 0 ? chans : INT32_MAX, cfg->mem_budget_bytes / per_chan);
    if (chans < 1) return XENG_ENOMEM;
    if (chans > 65536) return XENG_EINVAL;

    auto *s = new (std::nothrow) xeng_server;
    if (!s) return XENG_ENOMEM;
    s->cfg = *cfg;
    s->cfg.max_channels = (int32_t)chans;
    s->frame_bytes = frame_bytes;
    s->out_i32 = out_bytes / 4;
    xeng_config c{cfg->n_inputs, (int32_t)chans, cfg->device, cfg->flags & XENG_NIBBLE_RE_LOW, 0};
    int rc = xeng_create(&c, &s->ctx);
    if (rc != XENG_OK) {
        delete s;
        return rc;
    }
    if (hipSetDevice(cfg->device) != hipSuccess || hipMalloc(&s->d_out, (size_t)(out_bytes * chans)) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
        destroy_server(s);
        return XENG_ENOMEM;
    }
    for (int32_t k = (int32_t)chans - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->slot_owner.assign((size_t)chans, -1);
    *out = s;
    return XENG_OK;
}

int xeng_server_destroy(xeng_server *s)
{
    if (!s) return XENG_EINVAL;
    (void)hipSetDevice(s->cfg.device);
    destroy_server(s);
    return XENG_OK;
}

int32_t xeng_server_max_channels(const xeng_server *s) { return s ? s->cfg.max_channels : -1; }

int xeng_server_admit(xeng_server *s, const uint8_t *frames, int64_t n_frames, int32_t host_frames,
                      double start_s, int64_t total_frames, int32_t *channel)
{
    if (!s || !frames || n_frames < 1 || start_s < 0 || total_frames < 0 || !channel ||
        (host_frames != 0 && host_frames != 1))
        return XENG_EINVAL;
    Chan c;
    c.src = frames;
    c.src_host = host_frames;
    c.src_frames = n_frames;
    c.start_s = start_s;
    c.total_frames = total_frames;
    if (host_frames) {
        if (hipSetDevice(s->cfg.device) != hipSuccess) return XENG_EDEVICE;
        if (hipMalloc(&c.ring, (size_t)(s->cfg.ring_frames * s->frame_bytes)) != hipSuccess) return XENG_ENOMEM;
    }
    if (!s->free_slots.empty()) {
        c.slot = s->free_slots.back();
        s->free_slots.pop_back();
        c.state = 1;
        c.phase = export_phase(s, c.slot);
        s->slot_owner[(size_t)c.slot] = (int32_t)s->chans.size();
    }
    s->chans.push_back(c);
    *channel = (int32_t)s->chans.size() - 1;
    return XENG_OK;
}

int xeng_server_run(xeng_server *s, double seconds, xeng_server_stats *stats)
{
    if (!s || seconds < 0 || !stats) return XENG_EINVAL;
    if (hipSetDevice(s->cfg.device) != hipSuccess) return XENG_EDEVICE;
    const xeng_server_config &cf = s->cfg;
    const int64_t n = cf.n_inputs;
    const int64_t tri = n * (n + 1) / 2;
    std::vector<float> lat;
    std::deque<InFlight> inflight;
    int64_t dropped = 0, launches = 0, frames_done = 0;
    const Clock::time_point t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    double next_launch = 0;
    int rc = XENG_OK;

    auto retire = [&](bool wait) -> int {
        while (!inflight.empty()) {
            InFlight &f = inflight.front();
            hipError_t q = wait ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
            if (q == hipErrorNotReady) return XENG_OK;
            if (q != hipSuccess) return XENG_EDEVICE;
            const double t = now_s();
            for (const Range &r : f.ranges) {
                Chan &c = s->chans[(size_t)r.chan];
                if (!r.skipped) {
                    for (int64_t fr = r.f0; fr < r.f1; ++fr)
                        lat.push_back((float)(1e3 * (t - release_time(s, c, fr))));
                    frames_done += r.f1 - r.f0;
                }
                c.done = r.f1;
                if (c.state == 1 && c.total_frames > 0 && c.done >= c.total_frames) {
                    // finished: zero what it integrated past its last export
                    // (queued behind that export) and free the slot
                    c.state = 2;
                    if (xeng_reset(s->ctx, c.slot, s->compute) != XENG_OK) return XENG_EDEVICE;
                    s->free_slots.push_back(c.slot);
                }
            }
            s->event_pool.push_back(f.ev);
            inflight.pop_front();
        }
        return XENG_OK;
    };

    while (rc == XENG_OK) {
        const double t = now_s();
        if (t >= seconds) break;
        // admissions into freed slots
        for (size_t k = 0; k < s->chans.size(); ++k) {
            Chan &c = s->chans[k];
            if (c.state == 0 && !s->free_slots.empty()) {
                c.slot = s->free_slots.back();
                s->free_slots.pop_back();
                c.state = 1;
                c.phase = export_phase(s, c.slot);
                s->slot_owner[(size_t)c.slot] = (int32_t)k;
                if (c.start_s < t) c.start_s = t;   // its stream starts once admitted
            }
        }
        // releases (and ingest copies for host sources)
        for (Chan &c : s->chans) {
            if (c.state != 1) continue;
            const int64_t limit = c.total_frames > 0 ? c.total_frames : INT64_MAX;
            while (c.released < limit && release_time(s, c, c.released) <= t) {
                const int64_t f = c.released++;
                if (!c.src_host) {
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
                const int64_t r = f % cf.ring_frames;
                if (hipMemcpyAsync(c.ring + r * s->frame_bytes, c.src + (f % c.src_frames) * s->frame_bytes,
                                   (size_t)s->frame_bytes, hipMemcpyHostToDevice, s->copy) != hipSuccess) {
                    rc = XENG_EDEVICE;
                    break;
                }
                hipEvent_t e = get_event(s);
                if (!e || hipEventRecord(e, s->copy) != hipSuccess) {
                    rc = XENG_EDEVICE;
                    break;
                }
                c.copies.push_back({f + 1, e});
            }
            while (!c.copies.empty()) {
                hipError_t q = hipEventQuery(c.copies.front().second);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    rc = XENG_EDEVICE;
                    break;
                }
                c.available = c.copies.front().first;
                s->event_pool.push_back(c.copies.front().second);
                c.copies.pop_front();
            }
        }
        if (rc != XENG_OK) break;
        if ((rc = retire(false)) != XENG_OK) break;
        // one batched launch over every channel's available frames
        if (t >= next_launch && (int)inflight.size() < cf.max_inflight) {
            std::vector<xeng_job> jobs;
            InFlight f;
            std::vector<int32_t> dump_now;
            for (size_t k = 0; k < s->chans.size(); ++k) {
                Chan &c = s->chans[k];
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
                        dump_now.push_back((int32_t)k);
                        continue;
                    }
                }
                if (c.available <= f0) continue;
                const int64_t wrap_n = c.src_host ? cf.ring_frames : c.src_frames;
                const int64_t wrap = (f0 / wrap_n + 1) * wrap_n;
                const int64_t next_gap = c.gaps.empty() ? INT64_MAX : c.gaps.front();
                const int64_t f1 = std::min({c.available, boundary, wrap, next_gap});
                const uint8_t *base = c.src_host ? c.ring + (f0 % cf.ring_frames) * s->frame_bytes
                                                 : c.src + (f0 % c.src_frames) * s->frame_bytes;
                xeng_job j;
                j.ctx = s->ctx;
                j.slot = c.slot;
                j.reserved = 0;
                j.d_samples = base;
                j.n_samples = (f1 - f0) * cf.frame_len;
                j.row_stride = n;
                jobs.push_back(j);
                f.ranges.push_back({(int32_t)k, f0, f1, false});
                c.launched = f1;
                if (f1 == boundary) dump_now.push_back((int32_t)k);
            }
            if (!f.ranges.empty()) {
                if (!jobs.empty() &&
                    (rc = xeng_correlate_batch(jobs.data(), (int32_t)jobs.size(), s->compute)) != XENG_OK)
                    break;
                // every export due after this launch, in two launches
                std::vector<xeng_dump_job> dj;
                dj.reserve(dump_now.size());
                for (int32_t k : dump_now) {
                    const Chan &c = s->chans[(size_t)k];
                    dj.push_back({s->ctx, c.slot, 1, s->d_out + (int64_t)c.slot * s->out_i32, 0, 0});
                }
                if ((rc = xeng_dump_batch(dj.data(), (int32_t)dj.size(), s->compute)) != XENG_OK) break;
                for (int32_t k : dump_now) {
                    Chan &c = s->chans[(size_t)k];
                    c.last_dump_first = std::max<int64_t>(0, c.launched - cf.dump_frames);
                    ++c.dumps;
                }
                f.ev = get_event(s);
                if (!f.ev || hipEventRecord(f.ev, s->compute) != hipSuccess) {
                    rc = XENG_EDEVICE;
                    break;
                }
                inflight.push_back(std::move(f));
                if (!jobs.empty()) ++launches;
                next_launch = t + cf.launch_period_us * 1e-6;
            }
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    const int rc2 = retire(true);
    if (rc == XENG_OK) rc = rc2;
    const double wall = now_s();
    std::memset(stats, 0, sizeof *stats);
    int64_t released = 0;
    for (const Chan &c : s->chans) released += c.released;
    stats->frames_released = released;
    stats->frames_done = frames_done;
    stats->frames_dropped = dropped;
    stats->launches = launches;
    for (const Chan &c : s->chans) stats->dumps += c.dumps;
    stats->seconds = wall;
    stats->tcmacs = (double)frames_done * cf.frame_len * (double)tri / wall / 1e12;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) { return (double)lat[std::min(lat.size() - 1, (size_t)(p * (double)lat.size()))]; };
        stats->p50_ms = pct(0.50);
        stats->p99_ms = pct(0.99);
        stats->max_ms = lat.back();
    }
    stats->backlog_frames = released - frames_done - dropped;
    return rc;
}

int xeng_server_channel_info(const xeng_server *s, int32_t channel, xeng_server_channel *info)
{
    if (!s || !info || channel < 0 || channel >= (int32_t)s->chans.size()) return XENG_EINVAL;
    const Chan &c = s->chans[(size_t)channel];
    info->state = c.state;
    info->slot = c.slot;
    info->frames_done = c.done;
    info->dumps = c.dumps;
    info->last_dump_first_frame = c.last_dump_first;
    return XENG_OK;
}

int xeng_server_last_dump(xeng_server *s, int32_t channel, int32_t *out)
{
    if (!s || !out || channel < 0 || channel >= (int32_t)s->chans.size()) return XENG_EINVAL;
    const Chan &c = s->chans[(size_t)channel];
    if (c.slot < 0 || c.dumps == 0) return XENG_EINVAL;
    if (s->slot_owner[(size_t)c.slot] != channel) return XENG_EBUSY;   // slot reused since
    if (hipSetDevice(s->cfg.device) != hipSuccess) return XENG_EDEVICE;
    if (hipStreamSynchronize(s->compute) != hipSuccess) return XENG_EDEVICE;
    if (hipMemcpy(out, s->d_out + (int64_t)c.slot * s->out_i32, (size_t)(s->out_i32 * 4), hipMemcpyDefault) !=
        hipSuccess)
        return XENG_EDEVICE;
    return XENG_OK;
}

}  // extern "C"
