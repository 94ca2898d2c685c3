// Host runtime and C ABI of the X-engine correlator: contexts and their
// device-resident accumulators, the integration-length guard, the plan cache
// and batched launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "../../include/xeng.h"
#include "xeng_internal.h"
#include "xeng_plan.h"

namespace xeng {
// The correlation kernels: general (128 x 128 tiles, any layout), wide
// (DMA, 128 x 256), narrow (N <= 64, time split over the waves), the
// general kernel's exact FP8 instance and the wide kernel's (the unsigned
// form, for batch jobs whose slot pre-sums are set up).
enum class Kind { General, Wide, Narrow, Fp8, WideFp8 };

hipError_t launch_correlate(const KernelArgs &a, int grid, bool aligned, hipStream_t stream);
hipError_t launch_correlate_unsigned(const KernelArgs &a, int grid, bool aligned, hipStream_t stream);
hipError_t launch_correlate_fp8(const KernelArgs &a, int grid, bool aligned, hipStream_t stream);
hipError_t launch_presum(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low, int32_t *sr,
                         int32_t *si, hipStream_t stream);
hipError_t launch_presum_correct(int32_t *acc, int n, int nt, int64_t n_samples, const int32_t *sr,
                                 const int32_t *si, hipStream_t stream);
hipError_t launch_correlate_dma(const KernelArgs &a, int grid, int waves, hipStream_t stream);
hipError_t launch_correlate_dma_unsigned(const KernelArgs &a, int grid, bool fp8, hipStream_t stream);
hipError_t launch_correlate_narrow(const KernelArgs &a, int grid, hipStream_t stream);
hipError_t init_dma_kernel();
hipError_t launch_dump(int32_t *acc, int32_t *diag, int n, int nt, int32_t *out, bool reset,
                       hipStream_t stream);
hipError_t launch_dump_batch(const DumpDesc *d_jobs, int n_jobs, int n_max, int nt_max, hipStream_t stream);
hipError_t launch_dump_corr(int32_t *acc, int32_t *diag, int n, int nt, int32_t *out, bool reset,
                            const int32_t *sums, int n4, int64_t t, int32_t *other, hipStream_t stream);
hipError_t launch_zero(int32_t *p, int64_t n_i32, hipStream_t stream);
hipError_t launch_pad_rows(const uint8_t *src, int64_t stride, int n, int64_t rows, int n16, uint8_t *dst,
                           hipStream_t stream);
hipError_t launch_reference(const uint8_t *s, int64_t n_samples, int n, int64_t stride,
                            uint32_t re_low, int32_t *out, hipStream_t stream);
hipError_t launch_batch_guard(const GuardJob *d_jobs, int n_jobs, int32_t *d_skip, int64_t *d_skipped,
                              hipStream_t stream);
hipError_t launch_set_count(int64_t *p, int64_t v, hipStream_t stream);
hipError_t static_scratch_address(void **ptr);
hipError_t init_beam_kernel();
double ceiling_macs(int grid, int iters);
int ceiling_threads();
hipError_t launch_mfma_ceiling(int grid, int iters, int32_t *out, int64_t *clk, bool stamp_start, bool stamp_end,
                               hipStream_t stream);
int64_t beam_image_bytes(int n);
void beam_image(const int8_t *w, int n, int n_beams, uint8_t *img);
hipError_t launch_beamform(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low,
                           const int8_t *d_w, int n_beams, int shift, void *out, int grid, hipStream_t stream);
hipError_t launch_sk_flags(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low,
                           int block_len, int64_t lo_num, int64_t hi_num, int64_t den, uint8_t *flags,
                           hipStream_t stream);
hipError_t launch_mask_rows(const uint8_t *src, int64_t stride, int n, int64_t rows, int n16, uint8_t *dst,
                            const uint8_t *flags, int block_len, int64_t t_first, hipStream_t stream);
hipError_t launch_counts(const uint8_t *flags, int nb, int n, int block_len, int last_len, uint32_t *bits,
                         int32_t *counts, hipStream_t stream);
hipError_t launch_counts_export(const int32_t *counts, int64_t npairs, int32_t base, int32_t *out,
                                hipStream_t stream);
hipError_t launch_static_plan(const SinglePlanArgs &a, Piece *pieces, int32_t *wg_off, int32_t used,
                              hipStream_t stream);
constexpr int64_t STATIC_SCRATCH_BYTES = INT64_C(1) << 20;
}  // namespace xeng

using namespace xeng;

namespace {

std::atomic<int> g_wgs_per_cu{2};      // general kernel
std::atomic<int> g_min_stages{4};
std::atomic<int> g_kernel{XENG_KERNEL_AUTO};
// Scratch bytes per padded chunk (single calls) and per batched call.
constexpr int64_t PAD_SCRATCH_DEFAULT = INT64_C(256) << 20;
std::atomic<int64_t> g_pad_bytes{PAD_SCRATCH_DEFAULT};
std::atomic<int> g_plan_order{XENG_PLAN_XCD};

// The plan of a launch: single jobs take the XCD-aware decomposition where
// it applies (and the order asks for it), everything else the linear
// stream-K plan.
Plan build_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages, TileShape shape, int order,
                int64_t cap = 0)
{
    if (cap > 0) return make_plan(jobs, n_jobs, max_wgs, min_stages, shape, cap);
    Plan p;
    if (order == XENG_PLAN_XCD && n_jobs == 1 && make_plan_xcd(jobs[0], max_wgs, shape, &p)) return p;
    return make_plan(jobs, n_jobs, max_wgs, min_stages, shape);
}

// Launch configuration of one call: the global settings, or what the
// autotuner found best for calls of the same job sizes.
struct Tuning {
    int kernel;       // XENG_KERNEL_*
    int wgs_per_cu;   // general kernel
    int min_stages;
    int order;        // XENG_PLAN_* of single-job launches
    int source;       // XENG_TUNE_*
    double us;        // measured time of a tuned entry (0: not measured)
};

Tuning global_tuning()
{
    return Tuning{g_kernel.load(), g_wgs_per_cu.load(), g_min_stages.load(), g_plan_order.load(), XENG_TUNE_SETTINGS,
                  0.0};
}

// Waves per workgroup of the DMA kernel instance a configuration launches.
int dma_waves(const Tuning &tu) { return tu.kernel == XENG_KERNEL_DMA4 ? 4 : 8; }

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct DevicePlan {
    Piece *d_pieces = nullptr;
    int32_t *d_off = nullptr;
    int32_t grid = 0;
};

// Staging of one batched launch: its job table and its plan, in one pinned
// host buffer copied to one device buffer; reused once the event recorded
// after its launch has completed.
struct JobTable {
    uint8_t *h = nullptr;   // pinned host staging
    uint8_t *d = nullptr;
    size_t cap = 0;         // bytes
    hipEvent_t ev = nullptr;
    bool pending = false;
};

constexpr int PLAN_CACHE_MAX = 64;
constexpr int JOB_RING = 8;

// Class of a call's jobs in the autotuner's table: the largest N, the
// power-of-two classes of the largest T and of the number of jobs, and
// whether any job can take the DMA kernel.  Calls of one class share a
// tuned configuration, so that a streaming server's launches, whose job
// counts and lengths vary from launch to launch, find one.
struct TuneClass {
    int32_t n = 0, t_class = 0, jobs_class = 0, dma = 0;
    std::string key() const
    {
        char b[64];
        std::snprintf(b, sizeof b, "%d/%d/%d/%d", n, t_class, jobs_class, dma);
        return b;
    }
};

int log2_floor(int64_t v)
{
    int k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}

TuneClass tune_class(const PlanJob *jobs, int n_jobs, bool any_dma)
{
    TuneClass c;
    int64_t t_max = 1;
    for (int j = 0; j < n_jobs; ++j) {
        c.n = std::max(c.n, jobs[j].n);
        t_max = std::max(t_max, jobs[j].t);
    }
    c.t_class = log2_floor(t_max);
    c.jobs_class = log2_floor(std::max(1, n_jobs));
    c.dma = any_dma ? 1 : 0;
    return c;
}

struct DeviceState {
    int device = 0;
    int cu_count = 0;
    uint8_t *d_zeros = nullptr;   // ZERO_BYTES zero samples (0x88) for the DMA kernel, then ZERO_BYTES of
                                  // the unsigned form's zero (0x00: nibbles u = 0, products of nothing)
    std::mutex mu;
    std::unordered_map<std::string, DevicePlan> plans;
    std::list<std::string> lru;
    // plans of batched calls, kept on the host only: every batched launch
    // copies its plan to the device with its job table, so that nothing in
    // that path allocates, frees or copies synchronously
    std::unordered_map<std::string, std::shared_ptr<const Plan>> host_plans;
    std::list<std::string> host_lru;
    JobTable ring[JOB_RING];
    int ring_next = 0;
    struct Tuned {
        TuneClass cls;
        Tuning tu;
    };
    std::unordered_map<std::string, Tuned> tuned;   // job class -> autotuned configuration
    std::atomic<int64_t *> clock{nullptr};             // xeng_clock_probe buffer
    hipMemPool_t pad_pool = nullptr;   // scratch of padded single-channel calls (keeps up to 1 GiB)
    uint8_t *static_scratch = nullptr;  // this device's copy of the fixed plan array (xeng_correlate_static)
};

std::mutex g_states_mu;
std::map<int, std::unique_ptr<DeviceState>> g_states;

// The device's architecture name ("gfx950"), without target features.
std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    return a;
}

// The tune-cache file of an architecture: $XENG_TUNE_DIR, else
// $XDG_CACHE_HOME/xeng, else $HOME/.cache/xeng, holding
// xeng_tune_<arch>.json.  Empty if none of them is set.
std::string tune_cache_path(const std::string &arch)
{
    std::string dir;
    const char *d = std::getenv("XENG_TUNE_DIR");
    const char *x = std::getenv("XDG_CACHE_HOME");
    const char *h = std::getenv("HOME");
    if (d && *d)
        dir = d;
    else if (x && *x)
        dir = std::string(x) + "/xeng";
    else if (h && *h)
        dir = std::string(h) + "/.cache/xeng";
    if (dir.empty() || arch.empty()) return "";
    return dir + "/xeng_tune_" + arch + ".json";
}

// One entry per line, so that the reader needs no JSON parser: the library
// writes every line in exactly this form.
constexpr const char *TUNE_LINE =
    "  {\"n\": %d, \"t_class\": %d, \"jobs_class\": %d, \"dma\": %d, \"kernel\": %d, \"wgs_per_cu\": %d, "
    "\"min_stages\": %d, \"plan_order\": %d, \"us_per_launch\": %lf}";

// The entries of the cache file at `path` written for `arch` (none if there
// is no such file); lines that do not parse or hold values out of range are
// skipped.
void read_tune_file(const std::string &path, const std::string &arch,
                    std::unordered_map<std::string, DeviceState::Tuned> *out)
{
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    bool arch_ok = false;
    const std::string head = "{\"arch\": \"" + arch + "\",";
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, head.c_str(), head.size()) == 0) {
            arch_ok = true;
            continue;
        }
        if (!arch_ok) continue;
        TuneClass c;
        Tuning tu{};
        double us = 0.0;
        if (std::sscanf(line, TUNE_LINE, &c.n, &c.t_class, &c.jobs_class, &c.dma, &tu.kernel, &tu.wgs_per_cu,
                        &tu.min_stages, &tu.order, &us) != 9)
            continue;
        if (c.n < 1 || c.t_class < 0 || c.t_class > 62 || c.jobs_class < 0 || c.jobs_class > 31 ||
            (c.dma != 0 && c.dma != 1) || tu.kernel < XENG_KERNEL_AUTO || tu.kernel > XENG_KERNEL_DMA4 ||
            tu.wgs_per_cu < 1 || tu.wgs_per_cu > 2 || tu.min_stages < 1 || tu.min_stages > (1 << 20) ||
            (tu.order != XENG_PLAN_LINEAR && tu.order != XENG_PLAN_XCD) || !(us >= 0.0))
            continue;
        tu.source = XENG_TUNE_CACHE_FILE;
        tu.us = us;
        (*out)[c.key()] = DeviceState::Tuned{c, tu};
    }
    std::fclose(f);
}

// Called once per device, at its first use.
void load_tune_cache(DeviceState *st)
{
    const std::string arch = arch_name(st->device);
    read_tune_file(tune_cache_path(arch), arch, &st->tuned);
}

// mkdir -p of the directory part of `path`.
bool make_parent_dirs(const std::string &path)
{
    for (size_t k = 1; k < path.size(); ++k) {
        if (path[k] != '/') continue;
        const std::string d = path.substr(0, k);
        if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return false;
    }
    return true;
}

// Writes the file's entries, updated by every tuned entry of `st`, back to
// its architecture's cache file (through a temporary file renamed over it,
// so that a reader never sees half a file).  Called with st->mu held.
// False if it could not.
bool save_tune_cache(DeviceState *st)
{
    const std::string arch = arch_name(st->device);
    const std::string path = tune_cache_path(arch);
    if (path.empty() || !make_parent_dirs(path)) return false;
    std::unordered_map<std::string, DeviceState::Tuned> all;
    read_tune_file(path, arch, &all);
    for (const auto &kv : st->tuned) all[kv.first] = kv.second;
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"arch\": \"%s\", \"format\": 1, \"entries\": [\n", arch.c_str());
    size_t k = 0;
    for (const auto &kv : all) {
        const TuneClass &c = kv.second.cls;
        const Tuning &tu = kv.second.tu;
        std::fprintf(f, TUNE_LINE, c.n, c.t_class, c.jobs_class, c.dma, tu.kernel, tu.wgs_per_cu, tu.min_stages,
                     tu.order, tu.us);
        std::fprintf(f, "%s\n", ++k < all.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fflush(f) == 0 && std::ferror(f) == 0;
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

DeviceState *device_state(int device)
{
    std::lock_guard<std::mutex> lk(g_states_mu);
    auto it = g_states.find(device);
    if (it != g_states.end()) return it->second.get();
    auto st = std::make_unique<DeviceState>();
    st->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        return nullptr;
    st->cu_count = cus;
    // zero samples that the DMA kernel reads in place of rows past a
    // piece's end; written once, before any launch that could read them
    if (hipMalloc(&st->d_zeros, 2 * ZERO_BYTES) != hipSuccess) return nullptr;
    void *scr = nullptr;
    if (hipMemset(st->d_zeros, 0x88, ZERO_BYTES) != hipSuccess ||
        hipMemset(st->d_zeros + ZERO_BYTES, 0x00, ZERO_BYTES) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        init_dma_kernel() != hipSuccess || init_beam_kernel() != hipSuccess ||
        static_scratch_address(&scr) != hipSuccess || !scr) {
        (void)hipFree(st->d_zeros);
        return nullptr;
    }
    st->static_scratch = static_cast<uint8_t *>(scr);
    load_tune_cache(st.get());
    DeviceState *p = st.get();
    g_states[device] = std::move(st);
    return p;
}

std::string plan_key(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages, TileShape shape, int order,
                     int64_t cap = 0)
{
    std::string k;
    k.reserve(40 + 16 * (size_t)n_jobs);
    k.append(reinterpret_cast<const char *>(&cap), sizeof cap);
    k.push_back(shape == TileShape::Wide ? 'w' : 's');
    k.push_back((char)('0' + order));
    k.append(reinterpret_cast<const char *>(&max_wgs), sizeof max_wgs);
    k.append(reinterpret_cast<const char *>(&min_stages), sizeof min_stages);
    for (int j = 0; j < n_jobs; ++j) {
        k.append(reinterpret_cast<const char *>(&jobs[j].n), sizeof jobs[j].n);
        k.append(reinterpret_cast<const char *>(&jobs[j].t), sizeof jobs[j].t);
    }
    return k;
}

// Configuration for calls with these jobs.  Called with st->mu held.
Tuning tuning_for(DeviceState *st, const PlanJob *jobs, int n_jobs, bool any_dma)
{
    if (!st->tuned.empty()) {
        auto it = st->tuned.find(tune_class(jobs, n_jobs, any_dma).key());
        if (it != st->tuned.end()) return it->second.tu;
    }
    return global_tuning();
}

// Planner limits for a launch: workgroups and the minimum piece length.
// The DMA kernel holds one workgroup per CU (its LDS ring fills most of the
// CU); the general kernel fits two.
void plan_limits(const DeviceState *st, TileShape shape, const Tuning &tu, int *max_wgs, int *min_stages)
{
    const int per_cu = shape == TileShape::Square   ? std::max(1, tu.wgs_per_cu)
                       : shape == TileShape::Narrow ? NARROW_WGS_PER_CU
                                                    : 1;
    *max_wgs = st->cu_count * per_cu;
    *min_stages = std::max(1, tu.min_stages);
}

// The cached plan for this key, if any.  Called with st->mu held.
bool find_plan(DeviceState *st, const std::string &key, DevicePlan *out)
{
    auto it = st->plans.find(key);
    if (it == st->plans.end()) return false;
    st->lru.remove(key);
    st->lru.push_front(key);
    *out = it->second;
    return true;
}

// Upload `plan` and cache it under `key`.  Called with st->mu held and the
// device current.
int cache_plan(DeviceState *st, const std::string &key, const Plan &plan, DevicePlan *out)
{
    DevicePlan dp;
    dp.grid = plan.grid;
    if (plan.grid > 0) {
        if (hipMalloc(&dp.d_pieces, plan.pieces.size() * sizeof(Piece)) != hipSuccess)
            return XENG_ENOMEM;
        if (hipMalloc(&dp.d_off, plan.wg_off.size() * sizeof(int32_t)) != hipSuccess) {
            (void)hipFree(dp.d_pieces);
            return XENG_ENOMEM;
        }
        // synchronous copies: a plan is built once per shape
        if (hipMemcpy(dp.d_pieces, plan.pieces.data(), plan.pieces.size() * sizeof(Piece),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dp.d_off, plan.wg_off.data(), plan.wg_off.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(dp.d_pieces);
            (void)hipFree(dp.d_off);
            return XENG_EDEVICE;
        }
    }
    if ((int)st->plans.size() >= PLAN_CACHE_MAX) {
        // hipFree waits for the device, so no queued launch still reads it
        const std::string victim = st->lru.back();
        st->lru.pop_back();
        DevicePlan old = st->plans[victim];
        st->plans.erase(victim);
        if (old.d_pieces) (void)hipFree(old.d_pieces);
        if (old.d_off) (void)hipFree(old.d_off);
    }
    st->plans.emplace(key, dp);
    st->lru.push_front(key);
    *out = dp;
    return XENG_OK;
}

// Look up (or build, upload and cache) the plan for these job sizes.
// Called with st->mu held and the device current.
int get_plan(DeviceState *st, const PlanJob *jobs, int n_jobs, TileShape shape, const Tuning &tu,
             DevicePlan *out, int64_t cap = 0)
{
    int max_wgs, min_stages;
    plan_limits(st, shape, tu, &max_wgs, &min_stages);
    const std::string key = plan_key(jobs, n_jobs, max_wgs, min_stages, shape, tu.order, cap);
    if (find_plan(st, key, out)) return XENG_OK;
    return cache_plan(st, key, build_plan(jobs, n_jobs, max_wgs, min_stages, shape, tu.order, cap), out);
}

int map_err(hipError_t e)
{
    if (e == hipSuccess) return XENG_OK;
    if (e == hipErrorOutOfMemory) return XENG_ENOMEM;
    return XENG_EDEVICE;
}

}  // namespace

struct xeng_batch {
    struct Acct {
        xeng_ctx *ctx;
        int32_t slot;
        int64_t n;
    };
    // device: the guard table (one GuardJob per job with samples), then the
    // skip flag (int32) and the count of refused launches (int64)
    uint8_t *d_guard = nullptr;
    GuardJob *d_gjobs = nullptr;
    int32_t *d_skip = nullptr;
    int64_t *d_skipped = nullptr;
    int64_t skipped_seen = 0;
    bool bound = false;          // the jobs' slots count this batch in ctx->bound
    struct Launch {
        Kind kind;
        int waves;
        uint32_t flags_and;
        int32_t grid;
        JobDesc *d_jobs;
        Piece *d_pieces;
        int32_t *d_off;
    };
    int device = 0;
    const uint8_t *zeros = nullptr;
    std::vector<Acct> acct;
    std::vector<Launch> launches;
};

struct xeng_beams {
    int32_t device = 0;
    int32_t n = 0;
    int32_t n_beams = 0;
    uint32_t flags = 0;
    int32_t cu_count = 0;
    int64_t bytes = 0;           // operand-order image: one LDS load per chunk of inputs
    uint8_t *d_w = nullptr;
    uint8_t *h_w = nullptr;      // pinned staging of weight updates
    hipEvent_t ev = nullptr;
    bool pending = false;
};

struct xeng_ctx {
    int32_t n = 0;
    int32_t n_slots = 0;
    int32_t device = 0;
    uint32_t flags = 0;
    int32_t nt = 0;
    int64_t slot_i32 = 0;
    int32_t *d_acc = nullptr;    // n_slots accumulators, then n_slots diagonal stagings
    int32_t *d_diag = nullptr;
    int64_t *d_count = nullptr;  // per slot: samples integrated, kept on the device for prepared batches
    int32_t *d_counts = nullptr; // XENG_COUNTS: per slot, int32 [count_i32]: samples per pair from flagged calls
    int64_t count_i32 = 0;       // N(N+1)/2 rounded up to a multiple of 4
    std::vector<int64_t> acc_t;
    std::vector<int64_t> flagged_t;   // samples integrated by flagged calls (their counts are in d_counts)
    // the unsigned form (xeng_correlate_presum, FP8 calls on the wide
    // kernel): per slot two buffers of [SR | SI] (n4 = N rounded up to 4,
    // each); the current one sums the samples integrated that way since the
    // slot's correction was last applied, psum_t counts them.  The
    // correction is linear in (SR, SI, T), so it is applied once, before
    // the slot is next read or cleared.  A resetting export applies it in
    // its own kernels, clears the other buffer and makes it current (the one
    // it read is cleared by the next such export).
    int32_t *d_psum = nullptr;
    std::vector<int64_t> psum_t;
    std::vector<uint8_t> psum_cur;
    // live prepared batches naming each slot; while > 0 the slot's device
    // counter (advanced by the batches' device guard) is the true count and
    // acc_t is refreshed from it before any host-side check
    std::vector<int32_t> bound;
    DeviceState *st = nullptr;
};

namespace {

bool slot_ok(const xeng_ctx *c, int32_t slot) { return c && slot >= 0 && slot < c->n_slots; }

// Calls that queue work with host-side bookkeeping (the integration counter,
// staging buffers, pooled scratch) are refused while their stream is being
// captured: a replay would repeat the work without the bookkeeping.  Only
// xeng_batch_launch may be captured.
int refuse_capture(hipStream_t stream)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return XENG_EDEVICE;
    return cs == hipStreamCaptureStatusNone ? XENG_OK : XENG_ENOTSUP;
}

// A slot named by a live prepared batch: wait for the device and take the
// device counter (which the batches' guard advances on every launch and
// replay) as the host's count.  Device current.
int refresh_count(xeng_ctx *c, int32_t slot)
{
    if (c->bound[(size_t)slot] == 0) return XENG_OK;
    if (hipDeviceSynchronize() != hipSuccess) return XENG_EDEVICE;
    int64_t v = 0;
    if (hipMemcpy(&v, c->d_count + slot, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return XENG_EDEVICE;
    c->acc_t[(size_t)slot] = v;
    return XENG_OK;
}

// A reset of a slot also clears its per-pair sample counts (XENG_COUNTS).
hipError_t reset_counts(xeng_ctx *c, int32_t slot, hipStream_t stream)
{
    if (!c->d_counts || c->flagged_t[(size_t)slot] == 0) return hipSuccess;
    c->flagged_t[(size_t)slot] = 0;
    return launch_zero(c->d_counts + (int64_t)slot * c->count_i32, c->count_i32, stream);
}

// After an eager call changed a bound slot's count: the new value goes to
// the device counter in stream order.
hipError_t publish_count(xeng_ctx *c, int32_t slot, hipStream_t stream)
{
    if (c->bound[(size_t)slot] == 0) return hipSuccess;
    return launch_set_count(c->d_count + slot, c->acc_t[(size_t)slot], stream);
}

// `may_store`: the launch runs once (not a prepared batch), so a slot that
// holds zeros (nothing integrated since its last reset) may be written by
// plain stores.
JobDesc make_job(const xeng_ctx *c, int32_t slot, const uint8_t *d_samples, int64_t stride, bool may_store)
{
    JobDesc jd;
    jd.samples = d_samples;
    jd.acc = c->d_acc + (int64_t)slot * c->slot_i32;
    jd.stride = stride;
    jd.n = c->n;
    jd.nt = c->nt;
    jd.flags = 0;
    if (c->flags & XENG_NIBBLE_RE_LOW) jd.flags |= JOB_RE_LOW;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(d_samples);
    if ((stride % 8) == 0 && (addr % 8) == 0 && c->n % 8 == 0) jd.flags |= JOB_ALIGNED8;
    if ((stride % 16) == 0 && (addr % 16) == 0 && c->n % 16 == 0) jd.flags |= JOB_DMA;
    if (may_store && c->acc_t[(size_t)slot] == 0 && c->bound[(size_t)slot] == 0) jd.flags |= JOB_FRESH;
    jd.pad = 0;
    jd.presum = nullptr;
    return jd;
}

// Kernel choice for one job: the general kernel where the tuning asks for
// it or the job cannot be read by DMA, else the narrow kernel for N up to
// 64 and the wide DMA kernel above.

bool use_dma(uint32_t flags, const Tuning &tu)
{
    return tu.kernel != XENG_KERNEL_GENERAL && tu.kernel != XENG_KERNEL_FP8 && (flags & JOB_DMA);
}

Kind kind_of(const JobDesc &jd, const Tuning &tu)
{
    // FP8: the wide kernel's instance of the unsigned form for jobs whose
    // caller set up the slot's pre-sums (eager batches), else the general
    // kernel's
    if (tu.kernel == XENG_KERNEL_FP8) return (jd.flags & JOB_DMA) && jd.presum ? Kind::WideFp8 : Kind::Fp8;
    if (!use_dma(jd.flags, tu)) return Kind::General;
    return jd.n <= NARROW_MAX_N ? Kind::Narrow : Kind::Wide;
}

TileShape shape_of(Kind k)
{
    return k == Kind::Wide || k == Kind::WideFp8 ? TileShape::Wide
           : k == Kind::Narrow                   ? TileShape::Narrow
                                                 : TileShape::Square;
}

// Longest piece of a kernel, in stages (0: its shape's default).  The FP8
// instance's fp32 sums stay exact integers below 2^24: at most 128 per
// sample, so pieces below 2^17 samples.
constexpr int64_t MAX_PIECE_STAGES_FP8 = ((1 << 17) - 1) / STAGE;   // 2047 stages
int64_t cap_of(Kind k)
{
    return k == Kind::Fp8 ? MAX_PIECE_STAGES_FP8 : k == Kind::WideFp8 ? MAX_PIECE_STAGES_FP8_UNSIGNED : 0;
}

hipError_t launch(const KernelArgs &a, int32_t grid, Kind kind, int waves, uint32_t flags_and, hipStream_t stream)
{
    if (kind == Kind::Wide) return launch_correlate_dma(a, grid, waves, stream);
    if (kind == Kind::Narrow) return launch_correlate_narrow(a, grid, stream);
    if (kind == Kind::Fp8) return launch_correlate_fp8(a, grid, (flags_and & JOB_ALIGNED8) != 0, stream);
    if (kind == Kind::WideFp8) return launch_correlate_dma_unsigned(a, grid, true, stream);
    return launch_correlate(a, grid, (flags_and & JOB_ALIGNED8) != 0, stream);
}

// A single-channel call the DMA kernel cannot read in place (N not a
// multiple of 16, or a base or stride not a multiple of 16 bytes) with N of
// at least PAD_MIN_N: the samples are copied, in chunks of time rows, into
// stream-ordered scratch with rows of N rounded up to 16 bytes padded with
// zero samples, and each chunk is correlated from there by the DMA kernel
// (about twice the general kernel's rate for a copy that moves each sample
// twice).  Below PAD_MIN_N the general kernel's 128 x 128 tiles waste less.
constexpr int PAD_MIN_N = 256;

// The device's scratch pool for padded jobs, created on first use: a pool
// of the library's own that keeps up to 1 GiB between calls (the default
// pool returns its memory at every synchronization, and mapping it again
// costs more than the copy).  Called with st->mu held, device current.
int pad_pool(DeviceState *st, hipMemPool_t *out)
{
    if (!st->pad_pool) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = st->device;
        hipMemPool_t pool = nullptr;
        hipError_t e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return map_err(e);
        uint64_t keep = UINT64_C(1) << 30;
        if ((e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return map_err(e);
        }
        st->pad_pool = pool;
    }
    *out = st->pad_pool;
    return XENG_OK;
}

// Called with st->mu held and the device current; updates acc_t per chunk.
// With `flags` ([n_blocks][N], block_len samples per block), flagged samples
// become the zero sample in the copy.
int correlate_padded(xeng_ctx *ctx, int32_t slot, const uint8_t *samples, int64_t n_samples, int64_t stride,
                     const Tuning &tu, hipStream_t stream, const uint8_t *flags = nullptr, int block_len = 0)
{
    const int n16 = (ctx->n + 15) / 16 * 16;
    const int64_t rows = std::min<int64_t>(n_samples, std::max<int64_t>(STAGE, g_pad_bytes.load() / n16 / STAGE * STAGE));
    hipMemPool_t pool = nullptr;
    int prc = pad_pool(ctx->st, &pool);
    if (prc != XENG_OK) return prc;
    uint8_t *scratch = nullptr;
    hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&scratch), (size_t)(rows * n16), pool, stream);
    if (e != hipSuccess) return map_err(e);
    int rc = XENG_OK;
    for (int64_t t0 = 0; t0 < n_samples; t0 += rows) {
        const int64_t tc = std::min(rows, n_samples - t0);
        e = flags ? launch_mask_rows(samples + t0 * stride, stride, ctx->n, tc, n16, scratch, flags, block_len, t0,
                                     stream)
                  : launch_pad_rows(samples + t0 * stride, stride, ctx->n, tc, n16, scratch, stream);
        if (e != hipSuccess) {
            rc = map_err(e);
            break;
        }
        KernelArgs a{};
        a.job0 = make_job(ctx, slot, scratch, n16, true);
        a.job0.n = n16;                 // the padded inputs hold zero samples
        a.job0.flags |= JOB_DMA | JOB_ALIGNED8;
        a.jobs = nullptr;
        a.zeros = ctx->st->d_zeros;
        a.clock = ctx->st->clock.load();
        // the wide kernel, unless the tuning asks for the general one
        const bool dma = tu.kernel != XENG_KERNEL_GENERAL;
        PlanJob pj{ctx->n, tc};
        DevicePlan dp;
        if ((rc = get_plan(ctx->st, &pj, 1, dma ? TileShape::Wide : TileShape::Square, tu, &dp)) != XENG_OK) break;
        a.pieces = dp.d_pieces;
        a.wg_off = dp.d_off;
        if ((e = launch(a, dp.grid, dma ? Kind::Wide : Kind::General, dma_waves(tu), a.job0.flags, stream)) !=
            hipSuccess) {
            rc = map_err(e);
            break;
        }
        ctx->acc_t[(size_t)slot] += tc;
    }
    e = hipFreeAsync(scratch, stream);
    if (rc == XENG_OK && e != hipSuccess) rc = map_err(e);
    e = publish_count(ctx, slot, stream);
    if (rc == XENG_OK && e != hipSuccess) rc = map_err(e);
    return rc;
}

// Validated jobs of a batch that have work, in input order.
struct JobList {
    int device = -1;
    DeviceState *st = nullptr;
    std::vector<PlanJob> pj;
    std::vector<JobDesc> descs;
    std::vector<int32_t> idx;    // index into the caller's array
};

// Argument checks shared by the batched calls.  `launches` > 0 also applies
// the integration guard for that many launches of every job.
int validate_jobs(const xeng_job *jobs, int32_t n_jobs, int64_t launches, bool may_store, JobList *out)
{
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return XENG_EINVAL;
    if (n_jobs == 0) return XENG_OK;
    if (!jobs[0].ctx) return XENG_EINVAL;
    const int device = jobs[0].ctx->device;
    std::set<std::pair<const xeng_ctx *, int32_t>> seen;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const xeng_job &j = jobs[k];
        if (!slot_ok(j.ctx, j.slot) || j.reserved != 0 || j.n_samples < 0 ||
            j.row_stride < j.ctx->n || j.row_stride > MAX_STRIDE ||
            (j.n_samples > 0 && !j.d_samples) || j.ctx->device != device)
            return XENG_EINVAL;
        if (j.n_samples > 0 && j.row_stride > INT64_MAX / j.n_samples) return XENG_EINVAL;
        if (!seen.insert({j.ctx, j.slot}).second) return XENG_EINVAL;
        if (launches > 0 && j.n_samples > 0 &&
            (j.n_samples > T_MAX / launches || j.n_samples * launches > T_MAX - j.ctx->acc_t[(size_t)j.slot]))
            return XENG_EOVERFLOW;
    }
    out->device = device;
    out->st = jobs[0].ctx->st;
    for (int32_t k = 0; k < n_jobs; ++k) {
        if (jobs[k].n_samples == 0) continue;
        out->pj.push_back(PlanJob{jobs[k].ctx->n, jobs[k].n_samples});
        out->descs.push_back(make_job(jobs[k].ctx, jobs[k].slot, jobs[k].d_samples, jobs[k].row_stride, may_store));
        out->idx.push_back(k);
    }
    return XENG_OK;
}

// One persistent launch: the jobs of a batch that take the same kernel.
struct Part {
    Kind kind = Kind::General;
    uint32_t flags_and = ~0u;
    std::vector<PlanJob> pj;
    std::vector<JobDesc> descs;
};

// Batched jobs the DMA kernel cannot read in place, with N >= PAD_MIN_N, are
// copied into one pooled scratch buffer (as many as fit in PAD_SCRATCH_BYTES,
// in job order; the rest keep the general kernel) and their descriptors
// point at the copy.  The caller frees *scratch on the stream after the
// launches.  Called with st->mu held and the device current.
int pad_batch_jobs(JobList &jl, const Tuning &tu, hipStream_t stream, uint8_t **scratch)
{
    *scratch = nullptr;
    // (FP8 jobs read in place: the general kernel's instance any array, the
    // wide kernel's the arrays it takes as they are)
    if (tu.kernel == XENG_KERNEL_GENERAL || tu.kernel == XENG_KERNEL_FP8) return XENG_OK;
    std::vector<size_t> pick;
    std::vector<int64_t> off;
    int64_t total = 0;
    for (size_t k = 0; k < jl.descs.size(); ++k) {
        const JobDesc &d = jl.descs[k];
        if ((d.flags & JOB_DMA) || d.n < PAD_MIN_N || jl.pj[k].t <= 0) continue;
        const int64_t bytes = jl.pj[k].t * (int64_t)((d.n + 15) / 16 * 16);
        if (total + bytes > g_pad_bytes.load()) continue;
        pick.push_back(k);
        off.push_back(total);
        total += (bytes + 255) / 256 * 256;
    }
    if (pick.empty()) return XENG_OK;
    hipMemPool_t pool = nullptr;
    int rc = pad_pool(jl.st, &pool);
    if (rc != XENG_OK) return rc;
    hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void **>(scratch), (size_t)total, pool, stream);
    if (e != hipSuccess) {
        *scratch = nullptr;
        return map_err(e);
    }
    for (size_t i = 0; i < pick.size(); ++i) {
        JobDesc &d = jl.descs[pick[i]];
        const int n16 = (d.n + 15) / 16 * 16;
        uint8_t *dst = *scratch + off[i];
        if ((e = launch_pad_rows(d.samples, d.stride, d.n, jl.pj[pick[i]].t, n16, dst, stream)) != hipSuccess)
            return map_err(e);
        d.samples = dst;
        d.stride = n16;
        d.n = n16;   // the padded inputs hold zero samples
        d.flags |= JOB_DMA;
    }
    return XENG_OK;
}

bool any_dma_job(const JobList &jl)
{
    for (const JobDesc &jd : jl.descs)
        if (jd.flags & JOB_DMA) return true;
    return false;
}

std::vector<Part> split_by_kernel(const JobList &jl, const Tuning &tu)
{
    Part by_kind[5];
    by_kind[(int)Kind::Wide].kind = Kind::Wide;
    by_kind[(int)Kind::Narrow].kind = Kind::Narrow;
    by_kind[(int)Kind::Fp8].kind = Kind::Fp8;
    by_kind[(int)Kind::WideFp8].kind = Kind::WideFp8;
    for (size_t k = 0; k < jl.descs.size(); ++k) {
        Part &p = by_kind[(int)kind_of(jl.descs[k], tu)];
        p.pj.push_back(jl.pj[k]);
        p.descs.push_back(jl.descs[k]);
        p.flags_and &= jl.descs[k].flags;
    }
    std::vector<Part> parts;
    for (Kind k : {Kind::Wide, Kind::Narrow, Kind::General, Kind::Fp8, Kind::WideFp8})
        if (!by_kind[(int)k].descs.empty()) parts.push_back(std::move(by_kind[(int)k]));
    return parts;
}

// The next staging buffer of the ring, at least `bytes` long, once the
// launch that last used it has completed.  Called with st->mu held and the
// device current.
int ring_acquire(DeviceState *st, size_t bytes, JobTable **out)
{
    JobTable &tb = st->ring[st->ring_next];
    st->ring_next = (st->ring_next + 1) % JOB_RING;
    hipError_t e = hipSuccess;
    if (tb.pending) {
        e = hipEventSynchronize(tb.ev);
        if (e != hipSuccess) return map_err(e);
        tb.pending = false;
    }
    if (!tb.ev && (e = hipEventCreateWithFlags(&tb.ev, hipEventDisableTiming)) != hipSuccess) return map_err(e);
    if (tb.cap < bytes) {
        if (tb.h) (void)hipHostFree(tb.h);
        if (tb.d) (void)hipFree(tb.d);
        tb.h = nullptr;
        tb.d = nullptr;
        tb.cap = 0;
        const size_t cap = std::max<size_t>(bytes + bytes / 2, 64 * sizeof(JobDesc));
        if ((e = hipHostMalloc(&tb.h, cap, hipHostMallocDefault)) != hipSuccess) return map_err(e);
        if ((e = hipMalloc(&tb.d, cap)) != hipSuccess) {
            (void)hipHostFree(tb.h);
            tb.h = nullptr;
            return map_err(e);
        }
        tb.cap = cap;
    }
    *out = &tb;
    return XENG_OK;
}

// Launch the parts of a batch, staging each job table through the ring.
// Every plan and staging buffer is obtained, and every table written into
// its pinned buffer, before the first copy or launch is queued: a host-side
// failure (ENOMEM, a failed wait for a ring buffer) queues nothing.
// Called with st->mu held and the device current.
int run_parts(DeviceState *st, const std::vector<Part> &parts, const Tuning &tu, hipStream_t stream)
{
    struct Staged {
        JobTable *tb;
        size_t bytes;
        KernelArgs a;
        int32_t grid;
        Kind kind;
        int waves;
        uint32_t flags_and;
    };
    std::vector<Staged> staged;
    staged.reserve(parts.size());
    for (const Part &part : parts) {
        const TileShape shape = shape_of(part.kind);
        int max_wgs, min_stages;
        plan_limits(st, shape, tu, &max_wgs, &min_stages);
        const std::string key =
            plan_key(part.pj.data(), (int)part.pj.size(), max_wgs, min_stages, shape, tu.order, cap_of(part.kind));
        std::shared_ptr<const Plan> plan;
        auto it = st->host_plans.find(key);
        if (it != st->host_plans.end()) {
            plan = it->second;
            st->host_lru.remove(key);
            st->host_lru.push_front(key);
        } else {
            plan = std::make_shared<const Plan>(
                build_plan(part.pj.data(), (int)part.pj.size(), max_wgs, min_stages, shape, tu.order,
                           cap_of(part.kind)));
            if ((int)st->host_plans.size() >= PLAN_CACHE_MAX) {
                st->host_plans.erase(st->host_lru.back());
                st->host_lru.pop_back();
            }
            st->host_plans.emplace(key, plan);
            st->host_lru.push_front(key);
        }
        if (plan->grid <= 0) continue;
        // [job descriptors | pieces | workgroup offsets], 16-byte aligned parts
        auto up16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
        const size_t b_jobs = part.descs.size() * sizeof(JobDesc);
        const size_t b_pieces = plan->pieces.size() * sizeof(Piece);
        const size_t b_off = plan->wg_off.size() * sizeof(int32_t);
        const size_t o_pieces = up16(b_jobs), o_off = o_pieces + up16(b_pieces);
        const size_t bytes = o_off + b_off;
        JobTable *tbp = nullptr;
        const int rc = ring_acquire(st, bytes, &tbp);
        if (rc != XENG_OK) return rc;
        std::memcpy(tbp->h, part.descs.data(), b_jobs);
        std::memcpy(tbp->h + o_pieces, plan->pieces.data(), b_pieces);
        std::memcpy(tbp->h + o_off, plan->wg_off.data(), b_off);
        Staged sg;
        sg.tb = tbp;
        sg.bytes = bytes;
        sg.a = KernelArgs{};
        sg.a.jobs = reinterpret_cast<const JobDesc *>(tbp->d);
        // the unsigned form's zero sample is the nibble pair (0, 0)
        sg.a.zeros = part.kind == Kind::WideFp8 ? st->d_zeros + ZERO_BYTES : st->d_zeros;
        sg.a.clock = st->clock.load();
        sg.a.pieces = reinterpret_cast<const Piece *>(tbp->d + o_pieces);
        sg.a.wg_off = reinterpret_cast<const int32_t *>(tbp->d + o_off);
        sg.grid = plan->grid;
        sg.kind = part.kind;
        sg.waves = dma_waves(tu);
        sg.flags_and = part.flags_and;
        staged.push_back(sg);
    }
    for (Staged &sg : staged) {
        hipError_t e = hipMemcpyAsync(sg.tb->d, sg.tb->h, sg.bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch(sg.a, sg.grid, sg.kind, sg.waves, sg.flags_and, stream);
        if (e == hipSuccess) e = hipEventRecord(sg.tb->ev, stream);
        if (e != hipSuccess) return map_err(e);
        sg.tb->pending = true;
    }
    return XENG_OK;
}

// The unsigned form with pre-sums, called with st->mu held and the device
// current, the arguments checked and the guard passed: the wide kernel's
// unsigned instance where the array allows the DMA kernel (and the tuning
// does not ask for the general one), int8 or, with `fp8`, FP8 products,
// which also forms the pre-sums; else the general kernel's int8 instance
// after a pre-sum pass.
int64_t psum_n4(const xeng_ctx *c) { return ((int64_t)c->n + 3) / 4 * 4; }
// Buffer `which` (0, 1) of the slot's pre-sums: [SR | SI].
int32_t *psum_buf(const xeng_ctx *c, int32_t slot, int which)
{
    return c->d_psum + ((int64_t)slot * 2 + which) * 2 * psum_n4(c);
}

// The slot's pending unsigned-form correction (see xeng_ctx::d_psum) into
// its accumulators, and its sums cleared; stream-ordered, before anything
// reads the slot.  With `discard` (the slot is being cleared) only the
// sums are cleared.
hipError_t settle_presum(xeng_ctx *c, int32_t slot, hipStream_t stream, bool discard = false)
{
    if (c->psum_t[(size_t)slot] == 0) return hipSuccess;
    const int64_t n4 = psum_n4(c);
    int32_t *sums = psum_buf(c, slot, c->psum_cur[(size_t)slot]);
    hipError_t e = hipSuccess;
    if (!discard)
        e = launch_presum_correct(c->d_acc + (int64_t)slot * c->slot_i32, c->n, c->nt, c->psum_t[(size_t)slot], sums,
                                  sums + n4, stream);
    if (e == hipSuccess) e = launch_zero(sums, 2 * n4, stream);
    if (e == hipSuccess) c->psum_t[(size_t)slot] = 0;
    return e;
}

int correlate_unsigned(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples, int64_t row_stride,
                       const Tuning &tu, bool fp8, hipStream_t stream)
{
    const int64_t n4 = psum_n4(ctx);
    int32_t *sums = psum_buf(ctx, slot, ctx->psum_cur[(size_t)slot]);   // accumulated across calls
    PlanJob pj{ctx->n, n_samples};
    DevicePlan dp;
    KernelArgs a{};
    a.job0 = make_job(ctx, slot, d_samples, row_stride, true);
    const bool wide = (a.job0.flags & JOB_DMA) != 0 && tu.kernel != XENG_KERNEL_GENERAL;
    fp8 = fp8 && wide;
    int rc = wide ? get_plan(ctx->st, &pj, 1, TileShape::Wide, tu, &dp,
                             fp8 ? MAX_PIECE_STAGES_FP8_UNSIGNED : MAX_PIECE_STAGES_WIDE)
                  : get_plan(ctx->st, &pj, 1, TileShape::Square, tu, &dp, MAX_PIECE_STAGES_UNSIGNED);
    if (rc != XENG_OK) return rc;
    // the unsigned form's zero sample is the nibble pair (0, 0)
    a.zeros = ctx->st->d_zeros + ZERO_BYTES;
    a.pieces = dp.d_pieces;
    a.wg_off = dp.d_off;
    const uint32_t re_low = (ctx->flags & XENG_NIBBLE_RE_LOW) ? 1u : 0u;
    // the wide kernel's diagonal waves add the pre-sums as they go; the
    // general kernel's instance needs the pass over the samples
    hipError_t e = hipSuccess;
    if (wide) a.presum = sums;
    else e = launch_presum(d_samples, n_samples, ctx->n, row_stride, re_low, sums, sums + n4, stream);
    if (e == hipSuccess)
        e = wide ? launch_correlate_dma_unsigned(a, dp.grid, fp8, stream)
                 : launch_correlate_unsigned(a, dp.grid, (a.job0.flags & JOB_ALIGNED8) != 0, stream);
    if (e != hipSuccess) return map_err(e);
    ctx->acc_t[(size_t)slot] += n_samples;
    ctx->psum_t[(size_t)slot] += n_samples;
    return map_err(publish_count(ctx, slot, stream));
}

}  // namespace

namespace xeng {

// A context (see xeng_create).  With `stream` null its memory is zeroed and
// the device synchronized before it returns; otherwise the zeroing is queued
// on `stream` and nothing waits, so every use of the context must be
// ordered after it on that stream (the streaming server's slots).
int create_ctx(const xeng_config *cfg, hipStream_t stream, xeng_ctx **out)
{
    if (!cfg || !out) return XENG_EINVAL;
    *out = nullptr;
    if (cfg->n_inputs < 1 || cfg->n_inputs > 65535 || cfg->n_slots < 1 ||
        cfg->device < 0 || (cfg->flags & ~(XENG_NIBBLE_RE_LOW | XENG_COUNTS)) || cfg->mem_budget_bytes < 0)
        return XENG_EINVAL;
    const int64_t count_i32 = (cfg->flags & XENG_COUNTS) ? (tri64(cfg->n_inputs) + 3) / 4 * 4 : 0;
    const int64_t slot_bytes = (slot_i32(cfg->n_inputs) + diag_i32(cfg->n_inputs) + count_i32) * 4;
    if (slot_bytes > INT64_MAX / cfg->n_slots) return XENG_ENOMEM;
    const int64_t bytes = slot_bytes * cfg->n_slots;
    if (cfg->mem_budget_bytes > 0 && bytes > cfg->mem_budget_bytes) return XENG_ENOMEM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device >= ndev) return XENG_EDEVICE;

    DeviceGuard guard(cfg->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return XENG_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return XENG_ENOTSUP;
    DeviceState *st = device_state(cfg->device);
    if (!st) return XENG_EDEVICE;

    auto *c = new (std::nothrow) xeng_ctx;
    if (!c) return XENG_ENOMEM;
    c->n = cfg->n_inputs;
    c->n_slots = cfg->n_slots;
    c->device = cfg->device;
    c->flags = cfg->flags;
    c->nt = n_tiles_side(cfg->n_inputs);
    c->slot_i32 = slot_i32(cfg->n_inputs);
    c->acc_t.assign((size_t)cfg->n_slots, 0);
    c->flagged_t.assign((size_t)cfg->n_slots, 0);
    c->psum_t.assign((size_t)cfg->n_slots, 0);
    c->psum_cur.assign((size_t)cfg->n_slots, 0);
    c->bound.assign((size_t)cfg->n_slots, 0);
    c->count_i32 = count_i32;
    c->st = st;
    hipError_t e = hipMalloc(&c->d_acc, (size_t)bytes);
    if (e != hipSuccess) {
        delete c;
        return map_err(e);
    }
    // counters padded to a multiple of 16 bytes (the zero kernel's unit)
    const int64_t n_count = ((int64_t)cfg->n_slots + 1) / 2 * 2;
    if ((e = hipMalloc(&c->d_count, (size_t)n_count * sizeof(int64_t))) != hipSuccess) {
        (void)hipFree(c->d_acc);
        delete c;
        return map_err(e);
    }
    const int64_t psum_i32 = (int64_t)cfg->n_slots * 4 * (((int64_t)cfg->n_inputs + 3) / 4 * 4);
    if ((e = hipMalloc(&c->d_psum, (size_t)psum_i32 * 4)) != hipSuccess) {
        (void)hipFree(c->d_acc);
        (void)hipFree(c->d_count);
        delete c;
        return map_err(e);
    }
    c->d_diag = c->d_acc + (int64_t)cfg->n_slots * c->slot_i32;
    if (count_i32) c->d_counts = c->d_diag + (int64_t)cfg->n_slots * diag_i32(cfg->n_inputs);
    e = launch_zero(c->d_acc, bytes / 4, stream);
    if (e == hipSuccess) e = launch_zero(c->d_psum, psum_i32, stream);
    if (stream) {
        if (e == hipSuccess) e = launch_zero(reinterpret_cast<int32_t *>(c->d_count), 2 * n_count, stream);
    } else {
        if (e == hipSuccess) e = hipMemset(c->d_count, 0, (size_t)cfg->n_slots * sizeof(int64_t));
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        (void)hipFree(c->d_acc);
        (void)hipFree(c->d_count);
        (void)hipFree(c->d_psum);
        delete c;
        return map_err(e);
    }
    *out = c;
    return XENG_OK;
}

}  // namespace xeng

extern "C" {

int xeng_create(const xeng_config *cfg, xeng_ctx **out) { return create_ctx(cfg, nullptr, out); }

int xeng_destroy(xeng_ctx *ctx)
{
    if (!ctx) return XENG_EINVAL;
    int rc = XENG_OK;
    {
        DeviceGuard guard(ctx->device);
        if (ctx->d_acc && hipFree(ctx->d_acc) != hipSuccess) rc = XENG_EDEVICE;
        if (ctx->d_count && hipFree(ctx->d_count) != hipSuccess) rc = XENG_EDEVICE;
        if (ctx->d_psum && hipFree(ctx->d_psum) != hipSuccess) rc = XENG_EDEVICE;
    }
    delete ctx;
    return rc;
}

int xeng_correlate(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                   int64_t row_stride, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || n_samples < 0 || row_stride < ctx->n || row_stride > MAX_STRIDE)
        return XENG_EINVAL;
    if (n_samples > 0 && !d_samples) return XENG_EINVAL;
    // sample offsets t * row_stride must stay addressable
    if (n_samples > 0 && row_stride > INT64_MAX / n_samples) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    if ((rc = refresh_count(ctx, slot)) != XENG_OK) return rc;
    if (n_samples > T_MAX - ctx->acc_t[(size_t)slot]) return XENG_EOVERFLOW;
    if (n_samples == 0) return XENG_OK;

    PlanJob pj{ctx->n, n_samples};
    DevicePlan dp;
    KernelArgs a{};
    a.job0 = make_job(ctx, slot, d_samples, row_stride, true);
    a.jobs = nullptr;
    a.zeros = ctx->st->d_zeros;
    a.clock = ctx->st->clock.load();
    // held through the launch so that no other thread evicts the plan first
    std::lock_guard<std::mutex> lk(ctx->st->mu);
    const Tuning tu = tuning_for(ctx->st, &pj, 1, (a.job0.flags & JOB_DMA) != 0);
    // FP8 on an array the DMA kernel reads: the unsigned form's FP8 products
    // on the wide kernel, whose stored nibbles are E4M3 codes as they stand
    if (tu.kernel == XENG_KERNEL_FP8 && (a.job0.flags & JOB_DMA))
        return correlate_unsigned(ctx, slot, d_samples, n_samples, row_stride, tu, true, stream);
    const Kind kind = kind_of(a.job0, tu);
    if (kind == Kind::General && tu.kernel != XENG_KERNEL_GENERAL && ctx->n >= PAD_MIN_N)
        return correlate_padded(ctx, slot, d_samples, n_samples, row_stride, tu, stream);
    rc = get_plan(ctx->st, &pj, 1, shape_of(kind), tu, &dp, cap_of(kind));
    if (rc != XENG_OK) return rc;
    a.pieces = dp.d_pieces;
    a.wg_off = dp.d_off;
    hipError_t e = launch(a, dp.grid, kind, dma_waves(tu), a.job0.flags, stream);
    if (e != hipSuccess) return map_err(e);
    ctx->acc_t[(size_t)slot] += n_samples;
    return map_err(publish_count(ctx, slot, stream));
}

int xeng_rfi_flags(const uint8_t *d_samples, int64_t n_samples, int32_t n_inputs, int64_t row_stride,
                   uint32_t flags, const xeng_rfi_config *cfg, uint8_t *d_flags, void *hip_stream)
{
    if (!cfg || n_inputs < 1 || n_samples < 0 || row_stride < n_inputs || row_stride > MAX_STRIDE ||
        (flags & ~XENG_NIBBLE_RE_LOW) || cfg->block_len < 2 || cfg->block_len > XENG_RFI_MAX_BLOCK ||
        cfg->den < 1 || cfg->den > 1024 || cfg->lo_num < 0 || cfg->hi_num < cfg->lo_num ||
        cfg->hi_num > 16 * cfg->den || cfg->reserved != 0)
        return XENG_EINVAL;
    if (n_samples == 0) return XENG_OK;
    if (!d_samples || !d_flags || row_stride > INT64_MAX / n_samples) return XENG_EINVAL;
    if ((n_samples + cfg->block_len - 1) / cfg->block_len > 65535) return XENG_EINVAL;   // grid y
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    return map_err(launch_sk_flags(d_samples, n_samples, n_inputs, row_stride, (flags & XENG_NIBBLE_RE_LOW) ? 1u : 0u,
                                   cfg->block_len, cfg->lo_num, cfg->hi_num, cfg->den, d_flags, stream));
}

int xeng_correlate_flagged(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                           int64_t row_stride, const uint8_t *d_flags, int32_t block_len, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || n_samples < 0 || row_stride < ctx->n || row_stride > MAX_STRIDE || block_len < 1 ||
        !ctx->d_counts)
        return XENG_EINVAL;
    if (n_samples > 0 && (!d_samples || !d_flags || row_stride > INT64_MAX / n_samples)) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    if ((rc = refresh_count(ctx, slot)) != XENG_OK) return rc;
    if (n_samples > T_MAX - ctx->acc_t[(size_t)slot]) return XENG_EOVERFLOW;
    if (n_samples == 0) return XENG_OK;
    const int64_t nb = (n_samples + block_len - 1) / block_len;
    if (nb > INT32_MAX / 32) return XENG_EINVAL;
    const int last_len = (int)(n_samples - (nb - 1) * block_len);
    std::lock_guard<std::mutex> lk(ctx->st->mu);
    PlanJob pj{ctx->n, n_samples};
    const Tuning tu = tuning_for(ctx->st, &pj, 1, true);   // masked rows are padded for the DMA kernel
    // the counts' bit masks first (scratch), so that a failure to get it
    // queues nothing
    hipMemPool_t pool = nullptr;
    if ((rc = pad_pool(ctx->st, &pool)) != XENG_OK) return rc;
    uint32_t *bits = nullptr;
    const size_t bits_bytes = (size_t)ctx->n * (size_t)((nb + 31) / 32) * sizeof(uint32_t);
    hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&bits), bits_bytes, pool, stream);
    if (e != hipSuccess) return map_err(e);
    // visibilities of the masked samples (acc_t advances per chunk), then
    // the pair counts; after a device error the slot's contents are not
    // defined (reset it)
    rc = correlate_padded(ctx, slot, d_samples, n_samples, row_stride, tu, stream, d_flags, block_len);
    if (rc == XENG_OK) {
        e = launch_counts(d_flags, (int)nb, ctx->n, block_len, last_len, bits,
                          ctx->d_counts + (int64_t)slot * ctx->count_i32, stream);
        if (e == hipSuccess) ctx->flagged_t[(size_t)slot] += n_samples;
        rc = map_err(e);
    }
    e = hipFreeAsync(bits, stream);
    if (rc == XENG_OK && e != hipSuccess) rc = map_err(e);
    return rc;
}

int xeng_correlate_presum(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                          int64_t row_stride, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || n_samples < 0 || row_stride < ctx->n || row_stride > MAX_STRIDE)
        return XENG_EINVAL;
    if (n_samples > 0 && (!d_samples || row_stride > INT64_MAX / n_samples)) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    if ((rc = refresh_count(ctx, slot)) != XENG_OK) return rc;
    if (n_samples > T_MAX - ctx->acc_t[(size_t)slot]) return XENG_EOVERFLOW;
    if (n_samples == 0) return XENG_OK;
    std::lock_guard<std::mutex> lk(ctx->st->mu);
    PlanJob pj{ctx->n, n_samples};
    const JobDesc jd = make_job(ctx, slot, d_samples, row_stride, true);
    const Tuning tu = tuning_for(ctx->st, &pj, 1, (jd.flags & JOB_DMA) != 0);
    return correlate_unsigned(ctx, slot, d_samples, n_samples, row_stride, tu, tu.kernel == XENG_KERNEL_FP8, stream);
}

int xeng_dump_counts(xeng_ctx *ctx, int32_t slot, int32_t *out, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || !out || !ctx->d_counts) return XENG_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    if ((rc = refresh_count(ctx, slot)) != XENG_OK) return rc;
    // samples integrated without flags count for every pair
    const int64_t base = ctx->acc_t[(size_t)slot] - ctx->flagged_t[(size_t)slot];
    return map_err(launch_counts_export(ctx->d_counts + (int64_t)slot * ctx->count_i32, tri64(ctx->n), (int32_t)base,
                                        out, stream));
}

int xeng_correlate_static(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                          int64_t row_stride, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || n_samples < 0 || row_stride < ctx->n || row_stride > MAX_STRIDE)
        return XENG_EINVAL;
    if (n_samples > 0 && !d_samples) return XENG_EINVAL;
    if (n_samples > 0 && row_stride > INT64_MAX / n_samples) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    if ((rc = refresh_count(ctx, slot)) != XENG_OK) return rc;
    if (n_samples > T_MAX - ctx->acc_t[(size_t)slot]) return XENG_EOVERFLOW;
    if (n_samples == 0) return XENG_OK;

    DeviceState *st = ctx->st;
    const Tuning tu = global_tuning();   // no tuned-table lookup: it builds a key string
    KernelArgs a{};
    a.job0 = make_job(ctx, slot, d_samples, row_stride, true);
    const bool dma = use_dma(a.job0.flags, tu);
    const TileShape shape = dma ? TileShape::Wide : TileShape::Square;
    int max_wgs, min_stages;
    plan_limits(st, shape, tu, &max_wgs, &min_stages);
    int64_t np = 0, used = 0;
    const SinglePlanArgs pa = single_plan(ctx->n, n_samples, shape, max_wgs, min_stages, &np, &used);
    // [pieces | workgroup offsets] in the fixed array
    const int64_t off_at = (np * (int64_t)sizeof(Piece) + 255) / 256 * 256;
    if (off_at + (used + 1) * (int64_t)sizeof(int32_t) > STATIC_SCRATCH_BYTES) return XENG_ENOMEM;
    Piece *pieces = reinterpret_cast<Piece *>(st->static_scratch);
    int32_t *wg_off = reinterpret_cast<int32_t *>(st->static_scratch + off_at);
    hipError_t e = launch_static_plan(pa, pieces, wg_off, (int32_t)used, stream);
    if (e != hipSuccess) return map_err(e);
    a.jobs = nullptr;
    a.zeros = st->d_zeros;
    a.clock = st->clock.load();
    a.pieces = pieces;
    a.wg_off = wg_off;
    if ((e = launch(a, (int32_t)used, dma ? Kind::Wide : Kind::General, dma_waves(tu), a.job0.flags, stream)) !=
        hipSuccess)
        return map_err(e);
    ctx->acc_t[(size_t)slot] += n_samples;
    return map_err(publish_count(ctx, slot, stream));
}

int xeng_correlate_batch(const xeng_job *jobs, int32_t n_jobs, void *hip_stream)
{
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return XENG_EINVAL;
    if (n_jobs == 0) return XENG_OK;
    if (!jobs[0].ctx) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(jobs[0].ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    // slots of live prepared batches: their true counts first
    for (int32_t k = 0; k < n_jobs; ++k)
        if (slot_ok(jobs[k].ctx, jobs[k].slot) && jobs[k].ctx->device == jobs[0].ctx->device &&
            (rc = refresh_count(jobs[k].ctx, jobs[k].slot)) != XENG_OK)
            return rc;
    JobList jl;
    rc = validate_jobs(jobs, n_jobs, 1, true, &jl);
    if (rc != XENG_OK || jl.descs.empty()) return rc;
    std::lock_guard<std::mutex> lk(jl.st->mu);
    const Tuning tu = tuning_for(jl.st, jl.pj.data(), (int)jl.pj.size(), any_dma_job(jl));
    // FP8 on arrays the wide kernel reads in place: its instance of the
    // unsigned form, adding into the slot's current pre-sums (the
    // correction follows at the slot's export)
    if (tu.kernel == XENG_KERNEL_FP8)
        for (size_t d = 0; d < jl.descs.size(); ++d)
            if (jl.descs[d].flags & JOB_DMA) {
                const xeng_job &j = jobs[jl.idx[d]];
                jl.descs[d].presum = psum_buf(j.ctx, j.slot, j.ctx->psum_cur[(size_t)j.slot]);
            }
    uint8_t *scratch = nullptr;
    rc = pad_batch_jobs(jl, tu, stream, &scratch);
    if (rc == XENG_OK) rc = run_parts(jl.st, split_by_kernel(jl, tu), tu, stream);
    if (scratch) {
        const hipError_t e = hipFreeAsync(scratch, stream);
        if (rc == XENG_OK && e != hipSuccess) rc = map_err(e);
    }
    if (rc != XENG_OK) return rc;
    for (size_t d = 0; d < jl.descs.size(); ++d)
        if (jl.descs[d].presum) jobs[jl.idx[d]].ctx->psum_t[(size_t)jobs[jl.idx[d]].slot] += jobs[jl.idx[d]].n_samples;
    for (int32_t k : jl.idx) {
        jobs[k].ctx->acc_t[(size_t)jobs[k].slot] += jobs[k].n_samples;
        const hipError_t e = publish_count(jobs[k].ctx, jobs[k].slot, stream);
        if (e != hipSuccess) return map_err(e);
    }
    return XENG_OK;
}

int xeng_dump(xeng_ctx *ctx, int32_t slot, int32_t *out, int32_t reset, void *hip_stream)
{
    if (!slot_ok(ctx, slot) || !out) return XENG_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    int32_t *acc = ctx->d_acc + (int64_t)slot * ctx->slot_i32;
    int32_t *diag = ctx->d_diag + (int64_t)slot * diag_i32(ctx->n);
    hipError_t e = hipSuccess;
    if (reset && ctx->psum_t[(size_t)slot] > 0) {
        // the pending correction inside the export itself
        const int cur = ctx->psum_cur[(size_t)slot];
        e = launch_dump_corr(acc, diag, ctx->n, ctx->nt, out, true, psum_buf(ctx, slot, cur), (int)psum_n4(ctx),
                             ctx->psum_t[(size_t)slot], psum_buf(ctx, slot, 1 - cur), stream);
        if (e == hipSuccess) {
            ctx->psum_cur[(size_t)slot] = (uint8_t)(1 - cur);
            ctx->psum_t[(size_t)slot] = 0;
        }
    } else {
        e = settle_presum(ctx, slot, stream);
        if (e == hipSuccess) e = launch_dump(acc, diag, ctx->n, ctx->nt, out, reset != 0, stream);
    }
    if (e != hipSuccess) return map_err(e);
    if (reset) {
        ctx->acc_t[(size_t)slot] = 0;
        if ((e = reset_counts(ctx, slot, stream)) != hipSuccess) return map_err(e);
        return map_err(publish_count(ctx, slot, stream));
    }
    return XENG_OK;
}

int xeng_dump_batch(const xeng_dump_job *jobs, int32_t n_jobs, void *hip_stream)
{
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return XENG_EINVAL;
    if (n_jobs == 0) return XENG_OK;
    if (!jobs[0].ctx) return XENG_EINVAL;
    const int device = jobs[0].ctx->device;
    std::set<std::pair<const xeng_ctx *, int32_t>> seen;
    std::vector<DumpDesc> descs((size_t)n_jobs);
    for (int32_t k = 0; k < n_jobs; ++k) {
        const xeng_dump_job &j = jobs[k];
        if (!slot_ok(j.ctx, j.slot) || !j.out || (j.reset != 0 && j.reset != 1) || j.reserved != 0 ||
            j.ctx->device != device || !seen.insert({j.ctx, j.slot}).second)
            return XENG_EINVAL;
        DumpDesc &d = descs[(size_t)k];
        d.acc = j.ctx->d_acc + (int64_t)j.slot * j.ctx->slot_i32;
        d.diag = j.ctx->d_diag + (int64_t)j.slot * diag_i32(j.ctx->n);
        d.out = j.out;
        d.n = j.ctx->n;
        d.nt = j.ctx->nt;
        d.reset = j.reset;
        d.pad = 0;
    }
    DeviceGuard guard(device);
    if (!guard.ok) return XENG_EDEVICE;
    DeviceState *st = jobs[0].ctx->st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int crc = refuse_capture(stream);
    if (crc != XENG_OK) return crc;
    std::lock_guard<std::mutex> lk(st->mu);
    for (int32_t k = 0; k < n_jobs; ++k) {
        const hipError_t e = settle_presum(jobs[k].ctx, jobs[k].slot, stream);
        if (e != hipSuccess) return map_err(e);
    }
    constexpr int32_t CHUNK = 65535;   // grid z limit
    for (int32_t k0 = 0; k0 < n_jobs; k0 += CHUNK) {
        const int32_t m = std::min(CHUNK, n_jobs - k0);
        int n_max = 0, nt_max = 0;
        for (int32_t k = k0; k < k0 + m; ++k) {
            n_max = std::max(n_max, (int)descs[(size_t)k].n);
            nt_max = std::max(nt_max, (int)descs[(size_t)k].nt);
        }
        const size_t bytes = (size_t)m * sizeof(DumpDesc);
        JobTable *tb = nullptr;
        int rc = ring_acquire(st, bytes, &tb);
        if (rc != XENG_OK) return rc;
        std::memcpy(tb->h, descs.data() + k0, bytes);
        hipError_t e = hipMemcpyAsync(tb->d, tb->h, bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = launch_dump_batch(reinterpret_cast<const DumpDesc *>(tb->d), m, n_max, nt_max, stream);
        if (e == hipSuccess) e = hipEventRecord(tb->ev, stream);
        if (e != hipSuccess) return map_err(e);
        tb->pending = true;
    }
    for (int32_t k = 0; k < n_jobs; ++k)
        if (jobs[k].reset) {
            jobs[k].ctx->acc_t[(size_t)jobs[k].slot] = 0;
            hipError_t e = reset_counts(jobs[k].ctx, jobs[k].slot, stream);
            if (e == hipSuccess) e = publish_count(jobs[k].ctx, jobs[k].slot, stream);
            if (e != hipSuccess) return map_err(e);
        }
    return XENG_OK;
}

int xeng_reset(xeng_ctx *ctx, int32_t slot, void *hip_stream)
{
    if (!slot_ok(ctx, slot)) return XENG_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    hipError_t e = launch_zero(ctx->d_acc + (int64_t)slot * ctx->slot_i32, ctx->slot_i32, stream);
    if (e == hipSuccess) e = settle_presum(ctx, slot, stream, true);
    if (e == hipSuccess) e = reset_counts(ctx, slot, stream);
    if (e != hipSuccess) return map_err(e);
    ctx->acc_t[(size_t)slot] = 0;
    return map_err(publish_count(ctx, slot, stream));
}

int64_t xeng_samples_integrated(const xeng_ctx *ctx, int32_t slot)
{
    if (!slot_ok(ctx, slot)) return -1;
    if (ctx->bound[(size_t)slot] == 0) return ctx->acc_t[(size_t)slot];
    DeviceGuard guard(ctx->device);
    int64_t v = -1;
    if (!guard.ok || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&v, ctx->d_count + slot, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    return v;
}

int64_t xeng_max_integration(void) { return T_MAX; }

int64_t xeng_slot_bytes(int32_t n_inputs)
{
    if (n_inputs < 1) return -1;
    return (slot_i32(n_inputs) + diag_i32(n_inputs)) * 4;
}

int32_t xeng_n_inputs(const xeng_ctx *ctx) { return ctx ? ctx->n : -1; }
int32_t xeng_n_slots(const xeng_ctx *ctx) { return ctx ? ctx->n_slots : -1; }

const char *xeng_strerror(int status)
{
    switch (status) {
    case XENG_OK: return "ok";
    case XENG_EINVAL: return "invalid argument";
    case XENG_EOVERFLOW: return "integration length would exceed the exact int32 bound";
    case XENG_ENOMEM: return "out of device memory or over the memory budget";
    case XENG_EDEVICE: return "HIP runtime error or device fault";
    case XENG_EBUSY: return "resource busy";
    case XENG_ENOTSUP: return "not supported on this device";
    default: return "unknown status";
    }
}

int xeng_correlate_reference(const uint8_t *d_samples, int64_t n_samples, int32_t n_inputs,
                             int64_t row_stride, uint32_t flags, int32_t *d_out, void *hip_stream)
{
    if (!d_out || n_inputs < 1 || n_samples < 0 || row_stride < n_inputs ||
        (flags & ~XENG_NIBBLE_RE_LOW) || (n_samples > 0 && !d_samples))
        return XENG_EINVAL;
    if (n_samples > T_MAX) return XENG_EOVERFLOW;
    if (n_samples > 0 && row_stride > INT64_MAX / n_samples) return XENG_EINVAL;
    hipError_t e = launch_reference(d_samples, n_samples, n_inputs, row_stride,
                                    (flags & XENG_NIBBLE_RE_LOW) ? 1u : 0u, d_out,
                                    static_cast<hipStream_t>(hip_stream));
    return map_err(e);
}

int64_t xeng_plan_inspect(const int32_t *n_inputs, const int64_t *n_samples, int32_t n_jobs,
                          int32_t n_workgroups, int32_t min_stages, int32_t wide,
                          xeng_piece_info *out, int64_t cap)
{
    if (n_jobs < 0 || (n_jobs > 0 && (!n_inputs || !n_samples)) || n_workgroups < 1 || cap < 0 ||
        (cap > 0 && !out) || wide < 0 || wide > 2)
        return XENG_EINVAL;
    std::vector<PlanJob> pj((size_t)n_jobs);
    for (int32_t k = 0; k < n_jobs; ++k) {
        if (n_inputs[k] < 1 || n_samples[k] < 0 || n_samples[k] > T_MAX) return XENG_EINVAL;
        if (wide == 2 && n_inputs[k] > NARROW_MAX_N) return XENG_EINVAL;
        pj[(size_t)k] = PlanJob{n_inputs[k], n_samples[k]};
    }
    if (min_stages <= 0) min_stages = g_min_stages.load();
    const TileShape shape = wide == 1 ? TileShape::Wide : wide == 2 ? TileShape::Narrow : TileShape::Square;
    Plan plan = build_plan(pj.data(), n_jobs, n_workgroups, min_stages, shape, g_plan_order.load());
    const int64_t np = (int64_t)plan.pieces.size();
    for (int64_t k = 0; k < np && k < cap; ++k) {
        const Piece &p = plan.pieces[(size_t)k];
        xeng_piece_info &o = out[k];
        const int a = p.tile & 0xFFFF, b = (p.tile >> 16) & 0xFFFF;
        o.job = p.job;
        o.ti = a;
        o.tj = wide == 1 ? 2 * b : b;
        o.atomic = p.t1_atomic < 0 ? 1 : 0;
        o.t0 = p.t0;
        o.t1 = p.t1_atomic & 0x7FFFFFFF;
        o.workgroup = plan.piece_wg[(size_t)k];
        o.n_tiles = wide == 1 ? 2 : 1;
    }
    return np;
}

int64_t xeng_plan_inspect_static(int32_t n_inputs, int64_t n_samples, int32_t n_workgroups, int32_t min_stages,
                                 int32_t wide, xeng_piece_info *out, int64_t cap)
{
    if (n_inputs < 1 || n_samples < 1 || n_samples > T_MAX || n_workgroups < 1 || cap < 0 || (cap > 0 && !out) ||
        (wide != 0 && wide != 1))
        return XENG_EINVAL;
    if (min_stages <= 0) min_stages = g_min_stages.load();
    int64_t np = 0, used = 0;
    const SinglePlanArgs pa = single_plan(n_inputs, n_samples, wide ? TileShape::Wide : TileShape::Square,
                                          n_workgroups, min_stages, &np, &used);
    // the device kernel's emission, run on the host: pieces in order, a
    // unit cut into several pieces flagged atomic
    int64_t k = 0, unit_first = 0;
    auto close_unit = [&]() {
        if (k - unit_first > 1)
            for (int64_t q = unit_first; q < k && q < cap; ++q) out[q].atomic = 1;
        unit_first = k;
    };
    single_fill(pa, [&](int64_t w, int32_t ti, int32_t tj, int64_t s0, int64_t s1, int64_t kk) {
        if (kk == 0) close_unit();
        if (k < cap) {
            xeng_piece_info &o = out[k];
            o.job = 0;
            o.ti = ti;
            o.tj = wide ? 2 * tj : tj;
            o.atomic = 0;
            o.t0 = s0 * STAGE;
            o.t1 = std::min<int64_t>(s1 * STAGE, n_samples);
            o.workgroup = (int32_t)w;
            o.n_tiles = wide ? 2 : 1;
        }
        ++k;
    });
    close_unit();
    return np;
}

namespace {

// Releases the batch's slots: a slot no other live batch names takes its
// device counter's value as the host's count again.  Device current.
void unbind_slots(xeng_batch *b)
{
    if (!b->bound) return;
    bool synced = false;
    for (const auto &a : b->acct) {
        int32_t &bd = a.ctx->bound[(size_t)a.slot];
        if (bd == 1) {
            if (!synced) {
                (void)hipDeviceSynchronize();
                synced = true;
            }
            int64_t v = 0;
            if (hipMemcpy(&v, a.ctx->d_count + a.slot, sizeof v, hipMemcpyDeviceToHost) == hipSuccess)
                a.ctx->acc_t[(size_t)a.slot] = v;
        }
        if (bd > 0) --bd;
    }
    b->bound = false;
}

void free_batch(xeng_batch *b)
{
    unbind_slots(b);
    for (auto &l : b->launches) {
        if (l.d_jobs) (void)hipFree(l.d_jobs);
        if (l.d_pieces) (void)hipFree(l.d_pieces);
        if (l.d_off) (void)hipFree(l.d_off);
    }
    if (b->d_guard) (void)hipFree(b->d_guard);
    delete b;
}

}  // namespace

int xeng_batch_create(const xeng_job *jobs, int32_t n_jobs, xeng_batch **out)
{
    if (!out) return XENG_EINVAL;
    *out = nullptr;
    JobList jl;
    int rc = validate_jobs(jobs, n_jobs, 0, false, &jl);
    if (rc != XENG_OK) return rc;
    if (n_jobs == 0) return XENG_EINVAL;
    auto *b = new (std::nothrow) xeng_batch;
    if (!b) return XENG_ENOMEM;
    b->device = jobs[0].ctx->device;
    b->zeros = jobs[0].ctx->st->d_zeros;
    for (int32_t k : jl.idx) b->acct.push_back({jobs[k].ctx, jobs[k].slot, jobs[k].n_samples});
    if (jl.descs.empty()) {
        *out = b;
        return XENG_OK;
    }
    DeviceGuard guard(b->device);
    if (!guard.ok) {
        delete b;
        return XENG_EDEVICE;
    }
    Tuning tu;
    {
        std::lock_guard<std::mutex> lk(jl.st->mu);
        tu = tuning_for(jl.st, jl.pj.data(), (int)jl.pj.size(), any_dma_job(jl));
    }
    for (const Part &part : split_by_kernel(jl, tu)) {
        const TileShape shape = shape_of(part.kind);
        const int per_cu = shape == TileShape::Square   ? std::max(1, tu.wgs_per_cu)
                           : part.kind == Kind::Narrow ? NARROW_WGS_PER_CU
                                                       : 1;
        const Plan plan = build_plan(part.pj.data(), (int)part.pj.size(), jl.st->cu_count * per_cu,
                                     std::max(1, tu.min_stages), shape, tu.order, cap_of(part.kind));
        xeng_batch::Launch l{part.kind, dma_waves(tu), part.flags_and, plan.grid, nullptr, nullptr, nullptr};
        b->launches.push_back(l);
        xeng_batch::Launch &lb = b->launches.back();
        const size_t nj = part.descs.size() * sizeof(JobDesc);
        const size_t np = plan.pieces.size() * sizeof(Piece);
        const size_t no = plan.wg_off.size() * sizeof(int32_t);
        hipError_t e = hipMalloc(&lb.d_jobs, nj);
        if (e == hipSuccess) e = hipMalloc(&lb.d_pieces, std::max<size_t>(np, sizeof(Piece)));
        if (e == hipSuccess) e = hipMalloc(&lb.d_off, no);
        // synchronous uploads: a prepared batch is built once
        if (e == hipSuccess) e = hipMemcpy(lb.d_jobs, part.descs.data(), nj, hipMemcpyHostToDevice);
        if (e == hipSuccess && np) e = hipMemcpy(lb.d_pieces, plan.pieces.data(), np, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(lb.d_off, plan.wg_off.data(), no, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_batch(b);
            return map_err(e);
        }
    }
    // the device guard: [GuardJob per job | skip flag | refused launches]
    std::vector<GuardJob> gj;
    for (const auto &a : b->acct) gj.push_back(GuardJob{a.ctx->d_count + a.slot, a.n});
    const size_t gbytes = (gj.size() * sizeof(GuardJob) + 15) / 16 * 16;
    hipError_t e = hipMalloc(&b->d_guard, gbytes + 16);
    if (e == hipSuccess) e = hipMemcpy(b->d_guard, gj.data(), gj.size() * sizeof(GuardJob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_guard + gbytes, 0, 16);
    if (e != hipSuccess) {
        free_batch(b);
        return map_err(e);
    }
    b->d_gjobs = reinterpret_cast<GuardJob *>(b->d_guard);
    b->d_skip = reinterpret_cast<int32_t *>(b->d_guard + gbytes);
    b->d_skipped = reinterpret_cast<int64_t *>(b->d_guard + gbytes + 8);
    // bind the slots: a slot no live batch names yet starts its device
    // counter from the host's count (which includes work already queued)
    for (const auto &a : b->acct) {
        if (a.ctx->bound[(size_t)a.slot] == 0 &&
            (e = hipMemcpy(a.ctx->d_count + a.slot, &a.ctx->acc_t[(size_t)a.slot], sizeof(int64_t),
                           hipMemcpyHostToDevice)) != hipSuccess) {
            free_batch(b);
            return map_err(e);
        }
        a.ctx->bound[(size_t)a.slot]++;
        b->bound = true;
    }
    *out = b;
    return XENG_OK;
}

int xeng_batch_launch(xeng_batch *b, void *hip_stream)
{
    if (!b) return XENG_EINVAL;
    if (b->launches.empty()) return XENG_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(b->device);
    if (!guard.ok) return XENG_EDEVICE;
    DeviceState *bst = device_state(b->device);
    hipError_t e = launch_batch_guard(b->d_gjobs, (int)b->acct.size(), b->d_skip, b->d_skipped, stream);
    if (e != hipSuccess) return map_err(e);
    for (const auto &l : b->launches) {
        KernelArgs a{};
        a.jobs = l.d_jobs;
        a.pieces = l.d_pieces;
        a.wg_off = l.d_off;
        a.zeros = b->zeros;
        a.clock = bst ? bst->clock.load() : nullptr;
        a.skip = b->d_skip;
        if ((e = launch(a, l.grid, l.kind, l.waves, l.flags_and, stream)) != hipSuccess) return map_err(e);
    }
    return XENG_OK;
}

int xeng_batch_check(xeng_batch *b)
{
    if (!b) return XENG_EINVAL;
    if (!b->d_skipped) return XENG_OK;
    DeviceGuard guard(b->device);
    if (!guard.ok) return XENG_EDEVICE;
    int64_t v = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&v, b->d_skipped, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
        return XENG_EDEVICE;
    if (v > b->skipped_seen) {
        b->skipped_seen = v;
        return XENG_EOVERFLOW;
    }
    return XENG_OK;
}

int xeng_batch_destroy(xeng_batch *b)
{
    if (!b) return XENG_EINVAL;
    DeviceGuard guard(b->device);
    free_batch(b);
    return XENG_OK;
}

static void fill_tuning(const Tuning &tu, xeng_tuning *out)
{
    out->kernel = tu.kernel;
    out->wgs_per_cu = tu.wgs_per_cu;
    out->min_stages = tu.min_stages;
    out->plan_order = tu.order;
    out->us_per_launch = tu.us;
    out->source = tu.source;
    out->saved = 0;
}

int xeng_autotune(const xeng_job *jobs, int32_t n_jobs, int32_t iters, void *hip_stream, xeng_tuning *best)
{
    if (iters < 1 || iters > 1000) return XENG_EINVAL;
    JobList jl;
    int rc = validate_jobs(jobs, n_jobs, 0, false, &jl);
    if (rc != XENG_OK) return rc;
    if (jl.descs.empty()) return XENG_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard guard(jl.device);
    if (!guard.ok) return XENG_EDEVICE;
    if ((rc = refuse_capture(stream)) != XENG_OK) return rc;

    // the trials accumulate into accumulators of the library's own (one per
    // job, zeroed before every candidate), never into the callers' slots
    int64_t scratch_i32 = 0;
    std::vector<int64_t> off;
    for (int32_t k : jl.idx) {
        off.push_back(scratch_i32);
        scratch_i32 += jobs[k].ctx->slot_i32;
    }
    int32_t *scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, (size_t)scratch_i32 * sizeof(int32_t));
    if (e != hipSuccess) return map_err(e);
    for (size_t k = 0; k < jl.descs.size(); ++k) {
        jl.descs[k].acc = scratch + off[k];
        jl.descs[k].flags &= ~JOB_FRESH;
    }

    const bool any_dma = any_dma_job(jl);
    const bool single = jl.descs.size() == 1;
    std::vector<Tuning> cands;
    for (int ms : {1, 4, 16, 64})
        for (int order : {XENG_PLAN_XCD, XENG_PLAN_LINEAR}) {
            if (!single && order == XENG_PLAN_XCD) continue;   // batches always take the linear order
            if (any_dma)
                for (int kern : {XENG_KERNEL_AUTO, XENG_KERNEL_DMA4})
                    cands.push_back(Tuning{kern, 2, ms, order, XENG_TUNE_MEASURED, 0.0});
            for (int w : {1, 2}) cands.push_back(Tuning{XENG_KERNEL_GENERAL, w, ms, order, XENG_TUNE_MEASURED, 0.0});
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    Tuning best_t = cands[0];
    float best_us = -1.0f;
    std::lock_guard<std::mutex> lk(jl.st->mu);
    for (const Tuning &tu : cands) {
        if (e != hipSuccess) break;
        const std::vector<Part> parts = split_by_kernel(jl, tu);
        if ((e = launch_zero(scratch, scratch_i32, stream)) != hipSuccess) break;
        if ((rc = run_parts(jl.st, parts, tu, stream)) != XENG_OK) break;   // warm-up, plan upload
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
        for (int it = 0; it < iters && rc == XENG_OK; ++it) rc = run_parts(jl.st, parts, tu, stream);
        if (rc != XENG_OK) break;
        if ((e = hipEventRecord(e1, stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        const float us = 1000.0f * ms / (float)iters;
        if (best_us < 0.0f || us < best_us) {
            best_us = us;
            best_t = tu;
        }
    }
    // the trial launches read the job table ring and the scratch: wait for
    // them before freeing it
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    (void)hipFree(scratch);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != XENG_OK) return rc;
    if (e != hipSuccess) return map_err(e);
    best_t.us = best_us;
    const TuneClass cls = tune_class(jl.pj.data(), (int)jl.pj.size(), any_dma);
    jl.st->tuned[cls.key()] = DeviceState::Tuned{cls, best_t};
    const bool saved = save_tune_cache(jl.st);
    if (best) {
        fill_tuning(best_t, best);
        best->saved = saved ? 1 : 0;
    }
    return XENG_OK;
}

int xeng_tuning_lookup(const xeng_job *jobs, int32_t n_jobs, xeng_tuning *out)
{
    if (!out) return XENG_EINVAL;
    JobList jl;
    int rc = validate_jobs(jobs, n_jobs, 0, false, &jl);
    if (rc != XENG_OK) return rc;
    Tuning tu = global_tuning();
    if (!jl.descs.empty()) {
        std::lock_guard<std::mutex> lk(jl.st->mu);
        tu = tuning_for(jl.st, jl.pj.data(), (int)jl.pj.size(), any_dma_job(jl));
    }
    fill_tuning(tu, out);
    return XENG_OK;
}

int32_t xeng_tune_cache_path(int32_t device, char *buf, int32_t len)
{
    if (device < 0 || len < 0 || (len > 0 && !buf)) return XENG_EINVAL;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device >= n_dev) return XENG_EDEVICE;
    const std::string path = tune_cache_path(arch_name(device));
    if (path.empty()) return XENG_ENOTSUP;
    if (len > 0) {
        const size_t n = std::min(path.size(), (size_t)len - 1);
        std::memcpy(buf, path.data(), n);
        buf[n] = '\0';
    }
    return (int32_t)path.size();
}

int xeng_clock_probe(int32_t device, int64_t *dev_buf)
{
    if (device < 0) return XENG_EINVAL;
    DeviceGuard guard(device);
    if (!guard.ok) return XENG_EDEVICE;
    DeviceState *st = device_state(device);
    if (!st) return XENG_EDEVICE;
    st->clock.store(dev_buf);
    return XENG_OK;
}

int xeng_mfma_ceiling(int32_t device, int32_t ms, double *mac_per_s, double *sclk_ghz)
{
    if (device < 0 || ms < 10 || ms > 10000 || !mac_per_s || !sclk_ghz) return XENG_EINVAL;
    DeviceGuard guard(device);
    if (!guard.ok) return XENG_EDEVICE;
    DeviceState *st = device_state(device);
    if (!st) return XENG_EDEVICE;
    const int grid = st->cu_count;
    int32_t *d_out = nullptr;
    int64_t *d_clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&d_out, (size_t)grid * ceiling_threads() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_clk, 4 * sizeof(int64_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int iters = 256;
    float t_ms = 0.f;
    // one short launch sizes the rest at about 5 ms each
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch_mfma_ceiling(grid, iters, d_out, d_clk, false, false, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
    if (e == hipSuccess) {
        const double want = iters * 5.0 / std::max(1e-3, (double)t_ms);
        iters = (int)std::min(1 << 22, std::max(256, (int)want / 4 * 4));
        // the first half lets the clock settle under the load; the second is timed
        const int n = std::max(2, ms / 5), half = n / 2;
        for (int k = 0; k < half && e == hipSuccess; ++k)
            e = launch_mfma_ceiling(grid, iters, d_out, d_clk, false, false, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
        for (int k = half; k < n && e == hipSuccess; ++k)
            e = launch_mfma_ceiling(grid, iters, d_out, d_clk, k == half, k == n - 1, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
        int64_t clk[4] = {0, 0, 0, 0};
        if (e == hipSuccess) e = hipMemcpy(clk, d_clk, sizeof(clk), hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            *mac_per_s = ceiling_macs(grid, iters) * (n - half) / (t_ms / 1e3);
            *sclk_ghz = clk[3] > clk[1] ? (double)(clk[2] - clk[0]) / ((double)(clk[3] - clk[1]) / 1e8) / 1e9 : 0.0;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_out) (void)hipFree(d_out);
    if (d_clk) (void)hipFree(d_clk);
    return map_err(e);
}

int xeng_set_tuning(int32_t wgs_per_cu, int32_t min_stages, int32_t kernel)
{
    if (wgs_per_cu > 2 || kernel > XENG_KERNEL_FP8) return XENG_EINVAL;
    if (wgs_per_cu > 0) g_wgs_per_cu.store(wgs_per_cu);
    if (min_stages > 0) g_min_stages.store(min_stages);
    if (kernel >= 0) g_kernel.store(kernel);
    // explicit settings replace what the autotuner chose
    std::lock_guard<std::mutex> lk(g_states_mu);
    for (auto &kv : g_states) {
        std::lock_guard<std::mutex> lk2(kv.second->mu);
        kv.second->tuned.clear();
    }
    return XENG_OK;
}

int xeng_beams_create(int32_t n_inputs, int32_t n_beams, int32_t device, uint32_t flags, const int8_t *weights,
                      xeng_beams **out)
{
    if (!out) return XENG_EINVAL;
    *out = nullptr;
    if (n_inputs < 1 || n_inputs > 65535 || n_beams < 1 || n_beams > XENG_BEAMS_MAX || device < 0 ||
        (flags & ~XENG_NIBBLE_RE_LOW) || !weights)
        return XENG_EINVAL;
    const int64_t wbytes = (int64_t)n_beams * n_inputs * 2;
    for (int64_t k = 0; k < wbytes; ++k)
        if (weights[k] == INT8_MIN) return XENG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return XENG_EDEVICE;
    DeviceGuard guard(device);
    if (!guard.ok) return XENG_EDEVICE;
    DeviceState *st = device_state(device);
    if (!st) return XENG_EDEVICE;
    auto *bm = new (std::nothrow) xeng_beams;
    if (!bm) return XENG_ENOMEM;
    bm->device = device;
    bm->n = n_inputs;
    bm->n_beams = n_beams;
    bm->flags = flags;
    bm->bytes = beam_image_bytes(n_inputs);
    bm->cu_count = st->cu_count;
    hipError_t e = hipMalloc(&bm->d_w, (size_t)bm->bytes);
    if (e == hipSuccess) e = hipHostMalloc(&bm->h_w, (size_t)bm->bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bm->ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        beam_image(weights, n_inputs, n_beams, bm->h_w);
        e = hipMemcpy(bm->d_w, bm->h_w, (size_t)bm->bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)xeng_beams_destroy(bm);
        return map_err(e);
    }
    *out = bm;
    return XENG_OK;
}

int xeng_beams_set_weights(xeng_beams *bm, const int8_t *weights, void *hip_stream)
{
    if (!bm || !weights) return XENG_EINVAL;
    const int64_t wbytes = (int64_t)bm->n_beams * bm->n * 2;
    for (int64_t k = 0; k < wbytes; ++k)
        if (weights[k] == INT8_MIN) return XENG_EINVAL;
    DeviceGuard guard(bm->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    // the staging buffer is reused once the previous update's copy is done
    if (bm->pending && hipEventSynchronize(bm->ev) != hipSuccess) return XENG_EDEVICE;
    bm->pending = false;
    beam_image(weights, bm->n, bm->n_beams, bm->h_w);
    hipError_t e = hipMemcpyAsync(bm->d_w, bm->h_w, (size_t)bm->bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(bm->ev, stream);
    if (e != hipSuccess) return map_err(e);
    bm->pending = true;
    return XENG_OK;
}

int xeng_beamform(xeng_beams *bm, const uint8_t *d_samples, int64_t n_samples, int64_t row_stride, int32_t shift,
                  void *d_out, void *hip_stream)
{
    if (!bm || n_samples < 0 || row_stride < bm->n || row_stride > MAX_STRIDE || shift < -1 || shift > 24)
        return XENG_EINVAL;
    if (n_samples > 0 && (!d_samples || !d_out || row_stride > INT64_MAX / n_samples)) return XENG_EINVAL;
    if (n_samples == 0) return XENG_OK;
    DeviceGuard guard(bm->device);
    if (!guard.ok) return XENG_EDEVICE;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int rc = refuse_capture(stream);
    if (rc != XENG_OK) return rc;
    const int64_t blocks = (n_samples + 127) / 128;      // row blocks of the kernel
    const int grid = (int)std::min<int64_t>(blocks, bm->cu_count);
    return map_err(launch_beamform(d_samples, n_samples, bm->n, row_stride, (bm->flags & XENG_NIBBLE_RE_LOW) ? 1u : 0u,
                                   reinterpret_cast<const int8_t *>(bm->d_w), bm->n_beams, shift, d_out, grid,
                                   stream));
}

int xeng_beams_destroy(xeng_beams *bm)
{
    if (!bm) return XENG_EINVAL;
    DeviceGuard guard(bm->device);
    if (bm->pending) (void)hipEventSynchronize(bm->ev);
    if (bm->ev) (void)hipEventDestroy(bm->ev);
    if (bm->h_w) (void)hipHostFree(bm->h_w);
    int rc = XENG_OK;
    if (bm->d_w && hipFree(bm->d_w) != hipSuccess) rc = XENG_EDEVICE;
    delete bm;
    return rc;
}

int xeng_set_plan_order(int32_t order)
{
    if (order != XENG_PLAN_LINEAR && order != XENG_PLAN_XCD) return XENG_EINVAL;
    g_plan_order.store(order);
    return XENG_OK;
}

int xeng_set_pad_chunk_bytes(int64_t bytes)
{
    if (bytes < 0) return XENG_EINVAL;
    g_pad_bytes.store(bytes == 0 ? PAD_SCRATCH_DEFAULT : bytes);
    return XENG_OK;
}

}  // extern "C"
