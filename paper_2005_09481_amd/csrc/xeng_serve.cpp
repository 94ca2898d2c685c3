// Streaming correlation server: channels ingest frames at the instrument's
// sample rate, the device accumulators integrate them, and every channel
// exports its visibilities each `dump_frames` frames (Sec. 2.1: samples every
// 2.56 us per channel; integrated visibilities exported at a cadence).
//
// xeng_server_run drives the real-time loop of the scheduling core
// (xeng_sched.h: releases, ingest, continuous batching, export boundaries,
// admission, latency) on the calling thread.  This file is its executor on
// one device: the device memory of slots (accumulators and export buffer,
// allocated when a channel first takes the slot and kept for later
// channels) and of host sources' rings (kept for the next host source), the
// free device memory that admission weighs them against, copy streams for
// host frames (the due frames of every host source in one gather kernel per
// pass of the loop, the workgroups reading pinned host memory over PCIe,
// gathers taking the streams in turn; a source that is not verified pinned
// and 16-byte aligned is copied frame by frame instead, channel k on stream
// k % COPY_STREAMS), one compute stream for the batched correlation launches
// (xeng_correlate_batch), the exports due after each (xeng_dump_batch, into
// one device buffer per slot) and slot resets, and events for completion.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/xeng.h"
#include "xeng_sched.h"

namespace xeng {
int create_ctx(const xeng_config *cfg, hipStream_t stream, xeng_ctx **out);
hipError_t launch_gather_frames(const uint8_t *const *src, uint8_t *const *dst, int n, int64_t bytes,
                                hipStream_t stream);
}

namespace {

using Clock = std::chrono::steady_clock;

// Streams for host frames (gathers, and copies of the frames that cannot be
// gathered).  Copies alone, measured with 256-sample frames of N=2048 (512
// KiB copies): one stream sustained 24 host-sourced channels, four 40, eight
// fewer than four.
constexpr int COPY_STREAMS = 4;

// Device memory admission leaves free (for the library's plans and staging
// and for other users of the device).
constexpr int64_t MEM_RESERVE = INT64_C(512) << 20;

// A roctx range over a scope: the server's phases show up in a
// rocprofv3 --marker-trace beside the kernels they queue.
struct Range {
    explicit Range(const char *what) { roctxRangePush(what); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Device-side state of a channel (its scheduling state lives in the core).
struct ChanMem {
    const uint8_t *src = nullptr;  // [src_frames][frame_len][N], device or pinned host
    const uint8_t *src_dev = nullptr;  // host source the gather kernel reads: its device-visible address
    uint8_t *ring = nullptr;       // device ring of a host source (while it streams)
    int32_t *exports = nullptr;    // caller's export ring ([n_exports][N(N+1)/2][2]) or null
    int32_t n_exports = 0;
    int64_t issued = 0;            // exports queued into the caller's ring
};

}  // namespace

struct xeng_server {
    xeng_server_config cfg;
    xeng::sched::Scheduler *sch = nullptr;
    std::vector<xeng_ctx *> slot_ctx;    // per slot: its accumulators (a one-slot context), once used
    std::vector<int32_t *> slot_out;     // per slot: its export buffer, once used
    std::vector<uint8_t *> rings;        // every ring allocated
    std::vector<uint8_t *> free_rings;   // rings no channel holds
    int64_t out_i32 = 0;                 // per export buffer
    int64_t frame_bytes = 0;
    std::vector<ChanMem> mem;
    hipStream_t compute = nullptr;
    std::vector<hipStream_t> copy;       // COPY_STREAMS ingest streams
    std::vector<hipEvent_t> event_pool;  // recorded events no longer named by a token
    std::vector<hipEvent_t> tokens;      // token -> event (the copies of one gather share one)
    std::vector<int64_t> free_tokens;
    std::unordered_map<hipEvent_t, int> ev_refs;   // tokens naming each event
    // copies held for the next gather: sources, ring destinations, and the
    // event their tokens name (recorded after the gather)
    std::vector<const uint8_t *> g_src;
    std::vector<uint8_t *> g_dst;
    hipEvent_t g_ev = nullptr;
    int64_t g_next = 0;                  // gathers so far: the copy streams take them in turn
    int64_t gathered = 0;                // frames gathered in the current run
};

namespace {

// The scheduling core's executor on the server's device.
class HipExec : public xeng::sched::Executor {
public:
    explicit HipExec(xeng_server *s) : s_(s), t0_(Clock::now()) {}

    double now() override { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    void start() override { t0_ = Clock::now(); }

    int copy(const xeng::sched::Chan &c, int32_t chan, int64_t frame, int64_t *token) override
    {
        Range r("xeng server: ingest copy");
        const ChanMem &m = s_->mem[(size_t)chan];
        uint8_t *dst = m.ring + (frame % s_->cfg.ring_frames) * s_->frame_bytes;
        if (m.src_dev) {
            // held for this pass's gather
            if (!s_->g_ev) {
                if ((s_->g_ev = take_event()) == nullptr) return XENG_EDEVICE;
                s_->ev_refs[s_->g_ev] = 0;
            }
            s_->g_src.push_back(m.src_dev + (frame % c.src_frames) * s_->frame_bytes);
            s_->g_dst.push_back(dst);
            ++s_->ev_refs[s_->g_ev];
            *token = name(s_->g_ev);
            return XENG_OK;
        }
        const uint8_t *src = m.src + (frame % c.src_frames) * s_->frame_bytes;
        hipStream_t st = s_->copy[(size_t)chan % s_->copy.size()];
        if (hipMemcpyAsync(dst, src, (size_t)s_->frame_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return XENG_EDEVICE;
        return record(st, token);
    }

    // The copies held this pass: one gather kernel, then their shared
    // event.  Gathers take the copy streams in turn: a gather cannot start
    // while a correlation launch holds every CU, and those queued meanwhile
    // then run side by side (one stream held the ingest to 48 channels of
    // N=2048, four reach 56; holding copies back for larger gathers, which
    // keep more CUs from the next correlation launch, did worse).  A
    // channel's frames become available in order whatever order gathers
    // complete in: its copies are polled front first.
    int flush() override { return gather(); }

    int gather()
    {
        if (s_->g_src.empty()) return XENG_OK;
        Range r("xeng server: ingest gather");
        hipStream_t st = s_->copy[(size_t)(s_->g_next++ % (int64_t)s_->copy.size())];
        const hipError_t e = xeng::launch_gather_frames(s_->g_src.data(), s_->g_dst.data(), (int)s_->g_src.size(),
                                                        s_->frame_bytes, st);
        s_->gathered += (int64_t)s_->g_src.size();
        s_->g_src.clear();
        s_->g_dst.clear();
        hipEvent_t ev = s_->g_ev;
        s_->g_ev = nullptr;
        if (e != hipSuccess || hipEventRecord(ev, st) != hipSuccess) return XENG_EDEVICE;
        return XENG_OK;
    }

    int launch(const std::vector<xeng::sched::Job> &jobs, const std::vector<xeng::sched::Job> &exports,
               int64_t *token) override
    {
        Range r("xeng server: launch + exports");
        const xeng::sched::Config &cf = s_->sch->config();
        int rc = XENG_OK;
        if (!jobs.empty()) {
            std::vector<xeng_job> js;
            js.reserve(jobs.size());
            for (const xeng::sched::Job &j : jobs) {
                const xeng::sched::Chan &c = s_->sch->chans()[(size_t)j.chan];
                const ChanMem &m = s_->mem[(size_t)j.chan];
                const uint8_t *base = c.host ? m.ring + (j.f0 % cf.ring_frames) * s_->frame_bytes
                                             : m.src + (j.f0 % c.src_frames) * s_->frame_bytes;
                xeng_job x;
                x.ctx = s_->slot_ctx[(size_t)j.slot];
                x.slot = 0;
                x.reserved = 0;
                x.d_samples = base;
                x.n_samples = (j.f1 - j.f0) * cf.frame_len;
                x.row_stride = s_->cfg.n_inputs;
                js.push_back(x);
            }
            if ((rc = xeng_correlate_batch(js.data(), (int32_t)js.size(), s_->compute)) != XENG_OK) return rc;
        }
        if (!exports.empty()) {
            std::vector<xeng_dump_job> dj;
            dj.reserve(exports.size());
            for (const xeng::sched::Job &e : exports) {
                ChanMem &m = s_->mem[(size_t)e.chan];
                int32_t *dst = s_->slot_out[(size_t)e.slot];
                if (m.exports) dst = m.exports + (m.issued++ % m.n_exports) * s_->out_i32;
                dj.push_back({s_->slot_ctx[(size_t)e.slot], 0, 1, dst, 0, 0});
            }
            if ((rc = xeng_dump_batch(dj.data(), (int32_t)dj.size(), s_->compute)) != XENG_OK) return rc;
        }
        return record(s_->compute, token);
    }

    int64_t free_bytes() override
    {
        size_t free = 0, total = 0;
        if (hipMemGetInfo(&free, &total) != hipSuccess) return 0;
        return (int64_t)free;
    }

    int attach(const xeng::sched::Chan &c, int32_t chan, int32_t slot, bool new_slot, bool new_ring) override
    {
        Range r("xeng server: admit");
        if (new_slot) {
            xeng_config cc{s_->cfg.n_inputs, 1, s_->cfg.device, s_->cfg.flags & XENG_NIBBLE_RE_LOW, 0};
            xeng_ctx *ctx = nullptr;
            int32_t *out = nullptr;
            // zeroed on the compute stream, where every later use of the
            // slot is queued: no wait for the launches in flight
            const int rc = xeng::create_ctx(&cc, s_->compute, &ctx);
            if (rc != XENG_OK) return rc;
            if (hipMalloc(&out, (size_t)(s_->out_i32 * 4)) != hipSuccess) {
                (void)xeng_destroy(ctx);
                return XENG_ENOMEM;
            }
            s_->slot_ctx[(size_t)slot] = ctx;
            s_->slot_out[(size_t)slot] = out;
        }
        if (new_ring) {
            uint8_t *ring = nullptr;
            if (hipMalloc(&ring, (size_t)(s_->cfg.ring_frames * s_->frame_bytes)) != hipSuccess) {
                // leave nothing allocated: the core counts memory only for
                // channels it admits
                if (new_slot) {
                    (void)xeng_destroy(s_->slot_ctx[(size_t)slot]);
                    (void)hipFree(s_->slot_out[(size_t)slot]);
                    s_->slot_ctx[(size_t)slot] = nullptr;
                    s_->slot_out[(size_t)slot] = nullptr;
                }
                return XENG_ENOMEM;
            }
            s_->rings.push_back(ring);
            s_->free_rings.push_back(ring);
        }
        if (c.host) {
            s_->mem[(size_t)chan].ring = s_->free_rings.back();
            s_->free_rings.pop_back();
        }
        return XENG_OK;
    }

    int detach(const xeng::sched::Chan &c, int32_t chan, int32_t slot) override
    {
        Range r("xeng server: slot reset");
        if (c.host) {
            // every launch that read the ring has completed
            s_->free_rings.push_back(s_->mem[(size_t)chan].ring);
            s_->mem[(size_t)chan].ring = nullptr;
        }
        return xeng_reset(s_->slot_ctx[(size_t)slot], 0, s_->compute);
    }

    int poll(int64_t token, bool wait) override
    {
        hipEvent_t e = s_->tokens[(size_t)token];
        if (e == s_->g_ev) {
            // a copy still held for the gather (its event not yet recorded)
            if (!wait) return 0;
            const int rc = gather();
            if (rc != XENG_OK) return rc;
        }
        const hipError_t q = wait ? hipEventSynchronize(e) : hipEventQuery(e);
        if (q == hipErrorNotReady) return 0;
        return q == hipSuccess ? 1 : XENG_EDEVICE;
    }

    void release(int64_t token) override
    {
        hipEvent_t e = s_->tokens[(size_t)token];
        auto it = s_->ev_refs.find(e);
        if (it != s_->ev_refs.end() && --it->second == 0) {
            s_->ev_refs.erase(it);
            s_->event_pool.push_back(e);
        }
        s_->tokens[(size_t)token] = nullptr;
        s_->free_tokens.push_back(token);
    }

    void idle() override { std::this_thread::sleep_for(std::chrono::microseconds(20)); }

private:
    hipEvent_t take_event()
    {
        hipEvent_t e = nullptr;
        if (!s_->event_pool.empty()) {
            e = s_->event_pool.back();
            s_->event_pool.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            return nullptr;
        }
        return e;
    }

    int64_t name(hipEvent_t e)
    {
        int64_t k;
        if (!s_->free_tokens.empty()) {
            k = s_->free_tokens.back();
            s_->free_tokens.pop_back();
            s_->tokens[(size_t)k] = e;
        } else {
            k = (int64_t)s_->tokens.size();
            s_->tokens.push_back(e);
        }
        return k;
    }

    int record(hipStream_t stream, int64_t *token)
    {
        hipEvent_t e = take_event();
        if (!e) return XENG_EDEVICE;
        if (hipEventRecord(e, stream) != hipSuccess) {
            s_->event_pool.push_back(e);
            return XENG_EDEVICE;
        }
        s_->ev_refs[e] = 1;
        *token = name(e);
        return XENG_OK;
    }

    xeng_server *s_;
    Clock::time_point t0_;
};

// A host source the gather kernel may read in place: pinned host memory
// holding all its frames in one allocation, 16-byte aligned, with frames of
// a multiple of 16 bytes.  Returns its device-visible address, or null (the
// source is then copied frame by frame).
const uint8_t *gather_source(const xeng_server *s, const uint8_t *frames, int64_t n_frames)
{
    if (s->frame_bytes % 16 != 0 || s->frame_bytes >= (INT64_C(1) << 31) ||
        reinterpret_cast<uintptr_t>(frames) % 16 != 0 || n_frames > INT64_MAX / s->frame_bytes)
        return nullptr;
    // the caller's current device is restored on return
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(s->cfg.device) != hipSuccess) return nullptr;
    hipPointerAttribute_t at;
    void *start = nullptr;
    size_t size = 0;
    hipDeviceptr_t p = const_cast<uint8_t *>(frames);
    const bool ok = hipPointerGetAttributes(&at, frames) == hipSuccess && at.type == hipMemoryTypeHost &&
                    at.devicePointer &&
                    hipPointerGetAttribute(&start, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, p) == hipSuccess &&
                    hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, p) == hipSuccess;
    (void)hipSetDevice(prev);
    if (!ok) return nullptr;
    const uintptr_t lo = reinterpret_cast<uintptr_t>(start), hi = lo + size;
    const uintptr_t a = reinterpret_cast<uintptr_t>(frames);
    if (a < lo || a >= hi || (uint64_t)n_frames * (uint64_t)s->frame_bytes > hi - a) return nullptr;
    // the device view of `frames` itself (both fields name the same byte,
    // whether they are given for the allocation's start or for the pointer)
    const uint8_t *dev = static_cast<const uint8_t *>(at.devicePointer);
    if (at.hostPointer) dev += a - reinterpret_cast<uintptr_t>(at.hostPointer);
    return reinterpret_cast<uintptr_t>(dev) % 16 == 0 ? dev : nullptr;
}

void destroy_server(xeng_server *s)
{
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    for (hipStream_t c : s->copy)
        if (c) (void)hipStreamSynchronize(c);
    for (uint8_t *r : s->rings) (void)hipFree(r);
    // every event once: the copies of one gather share theirs
    std::unordered_set<hipEvent_t> evs(s->event_pool.begin(), s->event_pool.end());
    for (hipEvent_t e : s->tokens)
        if (e) evs.insert(e);
    if (s->g_ev) evs.insert(s->g_ev);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    for (hipStream_t c : s->copy)
        if (c) (void)hipStreamDestroy(c);
    for (int32_t *o : s->slot_out)
        if (o) (void)hipFree(o);
    for (xeng_ctx *c : s->slot_ctx)
        if (c) (void)xeng_destroy(c);
    delete s->sch;
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
    // device bytes of a slot (accumulators and export buffer) and of a host
    // source's ingest ring, allocated as channels are admitted
    const int64_t slot_bytes = xeng_slot_bytes(cfg->n_inputs) + out_bytes;
    const int64_t ring_bytes = (int64_t)cfg->ring_frames * frame_bytes;
    int64_t chans = cfg->max_channels;
    if (cfg->mem_budget_bytes > 0)
        chans = std::min<int64_t>(chans > 0 ? chans : INT32_MAX, cfg->mem_budget_bytes / slot_bytes);
    if (chans < 1) return XENG_ENOMEM;
    if (chans > 65536) return XENG_EINVAL;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || cfg->device >= n_dev) return XENG_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return XENG_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return XENG_ENOTSUP;

    auto *s = new (std::nothrow) xeng_server;
    if (!s) return XENG_ENOMEM;
    s->cfg = *cfg;
    s->cfg.max_channels = (int32_t)chans;
    s->frame_bytes = frame_bytes;
    s->out_i32 = out_bytes / 4;
    xeng::sched::Config sc;
    sc.frame_len = cfg->frame_len;
    sc.dump_frames = cfg->dump_frames;
    sc.ring_frames = cfg->ring_frames;
    sc.max_inflight = cfg->max_inflight;
    sc.slots = (int32_t)chans;
    sc.frame_period_us = cfg->frame_period_us;
    sc.launch_period_us = cfg->launch_period_us;
    sc.stagger_exports = (cfg->flags & XENG_SERVER_STAGGER_EXPORTS) != 0;
    sc.pairs = (double)(n * (n + 1) / 2);
    sc.slot_bytes = slot_bytes;
    sc.ring_bytes = ring_bytes;
    sc.mem_budget = cfg->mem_budget_bytes;
    sc.mem_reserve = MEM_RESERVE;
    s->sch = new (std::nothrow) xeng::sched::Scheduler(sc);
    if (!s->sch) {
        delete s;
        return XENG_ENOMEM;
    }
    s->slot_ctx.assign((size_t)chans, nullptr);
    s->slot_out.assign((size_t)chans, nullptr);
    bool ok = hipSetDevice(cfg->device) == hipSuccess &&
              hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; ok && k < COPY_STREAMS; ++k) {
        hipStream_t c = nullptr;
        ok = hipStreamCreateWithFlags(&c, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->copy.push_back(c);
    }
    if (!ok) {
        destroy_server(s);
        return XENG_EDEVICE;
    }
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
    ChanMem m;
    m.src = frames;
    if (host_frames) m.src_dev = gather_source(s, frames, n_frames);
    s->mem.push_back(m);
    *channel = s->sch->admit(n_frames, host_frames != 0, start_s, total_frames);
    return XENG_OK;
}

int xeng_server_run(xeng_server *s, double seconds, xeng_server_stats *stats)
{
    if (!s || seconds < 0 || !stats) return XENG_EINVAL;
    if (hipSetDevice(s->cfg.device) != hipSuccess) return XENG_EDEVICE;
    HipExec ex(s);
    xeng::sched::Stats st;
    int rc;
    s->gathered = 0;
    {
        Range r("xeng server: run");
        rc = s->sch->run(ex, seconds, &st);
        // nothing stays held for a gather between runs
        const int rf = ex.gather();
        if (rc == XENG_OK) rc = rf;
    }
    stats->frames_released = st.frames_released;
    stats->frames_done = st.frames_done;
    stats->frames_dropped = st.frames_dropped;
    stats->launches = st.launches;
    stats->dumps = st.dumps;
    stats->backlog_frames = st.backlog_frames;
    stats->channels_waiting = st.waiting;
    stats->device_bytes = st.device_bytes;
    stats->seconds = st.seconds;
    stats->tcmacs = st.tcmacs;
    stats->p50_ms = st.p50_ms;
    stats->p99_ms = st.p99_ms;
    stats->max_ms = st.max_ms;
    stats->max_pass_ms = st.max_pass_ms;
    stats->max_launch_call_ms = st.max_launch_call_ms;
    stats->max_copy_call_ms = st.max_copy_call_ms;
    stats->frames_gathered = s->gathered;
    return rc;
}

int xeng_server_channel_info(const xeng_server *s, int32_t channel, xeng_server_channel *info)
{
    if (!s || !info || channel < 0 || channel >= (int32_t)s->sch->chans().size()) return XENG_EINVAL;
    const xeng::sched::Chan &c = s->sch->chans()[(size_t)channel];
    info->state = c.state;
    info->slot = c.slot;
    info->frames_done = c.done;
    info->dumps = c.dumps;
    info->last_dump_first_frame = c.last_dump_first;
    info->admitted_s = c.admitted_s;
    return XENG_OK;
}

int xeng_server_last_dump(xeng_server *s, int32_t channel, int32_t *out)
{
    if (!s || !out || channel < 0 || channel >= (int32_t)s->sch->chans().size()) return XENG_EINVAL;
    const xeng::sched::Chan &c = s->sch->chans()[(size_t)channel];
    const ChanMem &m = s->mem[(size_t)channel];
    if (c.slot < 0 || c.dumps == 0) return XENG_EINVAL;
    const int32_t *src = nullptr;
    if (m.exports) {
        src = m.exports + ((m.issued - 1) % m.n_exports) * s->out_i32;
    } else {
        if (s->sch->slot_owner(c.slot) != channel) return XENG_EBUSY;   // slot reused since
        src = s->slot_out[(size_t)c.slot];
    }
    if (hipSetDevice(s->cfg.device) != hipSuccess) return XENG_EDEVICE;
    if (hipStreamSynchronize(s->compute) != hipSuccess) return XENG_EDEVICE;
    if (hipMemcpy(out, src, (size_t)(s->out_i32 * 4), hipMemcpyDefault) != hipSuccess) return XENG_EDEVICE;
    return XENG_OK;
}

int xeng_server_export_ring(xeng_server *s, int32_t channel, int32_t *ring, int32_t n_entries)
{
    if (!s || channel < 0 || channel >= (int32_t)s->sch->chans().size() || (ring && n_entries < 1) ||
        (!ring && n_entries != 0))
        return XENG_EINVAL;
    ChanMem &m = s->mem[(size_t)channel];
    if (m.issued != 0 || s->sch->chans()[(size_t)channel].dumps != 0) return XENG_EBUSY;
    m.exports = ring;
    m.n_exports = n_entries;
    return XENG_OK;
}

}  // extern "C"
