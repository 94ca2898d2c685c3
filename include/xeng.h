/*
 * xeng -- X-engine correlator for AMD MI355X (gfx950).  C ABI.
 *
 * The operation (Sec. 2.2, "Computational Requirements"; the per-channel
 * GPU task of Sec. 2.3 and Table tab:computing): for one frequency channel
 * of an N-input array, every time sample t carries one complex value per
 * input, 4 bits real + 4 bits imaginary.  The correlator forms, for every
 * pair 0 <= i <= j < N (the N(N+1)/2 products of the cost model eta,
 * autocorrelations included),
 *
 *         V_ij = sum_t x_i(t) * conj(x_j(t))
 *
 * and integrates it over time in exact int32 accumulators that live on the
 * device; the integrated visibilities are exported ("dumped") at a cadence
 * chosen by the caller (Sec. 2.1 and Sec. 3.1: visibilities leave the node
 * after substantial time integration).
 *
 * Sample format: one byte per complex sample; each part is offset-binary,
 * value = nibble - 8 (range -8..7); the real part is in the high nibble
 * unless XENG_NIBBLE_RE_LOW is set.  A flagged input is represented by the
 * zero sample, byte 0x88.  Sample arrays are time-major: sample t of input i
 * is at d_samples[t * row_stride + i], row_stride >= N.
 *
 * Visibility format (xeng_dump): int32 pairs (Re, Im), upper triangle row by
 * row: pair (i, j), i <= j, at index k = i*N - i*(i-1)/2 + (j - i); the
 * buffer holds N(N+1)/2 pairs = 4*N*(N+1) bytes.
 *
 * Exactness: every product has |Re| <= 128 and |Im| <= 120, so a slot can
 * integrate at most xeng_max_integration() = 16,777,215 samples between
 * dumps (128 * 16,777,215 <= 2^31 - 1).  Calls that would pass this bound
 * are refused with XENG_EOVERFLOW, whatever the data, and change nothing.
 *
 * Errors: every call returns a status (never throws across the ABI).
 * Argument, bound and budget errors are detected on the host before any
 * work is queued and leave all state unchanged.  Device-side faults are
 * reported as XENG_EDEVICE by the call that observes them.
 *
 * Streams: `hip_stream` is a hipStream_t (NULL = the default stream).  Work
 * is queued asynchronously; buffers passed in must stay valid until the
 * stream reaches the queued work.  Calls on one slot must be ordered on one
 * stream.  One context is not thread-safe; distinct contexts are.
 *
 * Graph capture: xeng_batch_launch is the one call that may be captured
 * into a hipGraph.  xeng_correlate, xeng_correlate_batch, xeng_dump,
 * xeng_dump_batch and xeng_reset keep host-side bookkeeping (the
 * integration counter, staging buffers, pooled scratch) that a replay would
 * not repeat, so they return XENG_ENOTSUP, queuing nothing, while their
 * stream is capturing.
 */
#ifndef XENG_H
#define XENG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XENG_ABI_VERSION 1

typedef struct xeng_ctx xeng_ctx;

enum xeng_status {
    XENG_OK = 0,
    XENG_EINVAL = -1,     /* bad argument (null pointer, size, slot, flags) */
    XENG_EOVERFLOW = -2,  /* integration would exceed xeng_max_integration() */
    XENG_ENOMEM = -3,     /* device allocation failed or exceeds mem_budget */
    XENG_EDEVICE = -4,    /* HIP runtime error or device fault */
    XENG_EBUSY = -5,      /* resource in use */
    XENG_ENOTSUP = -6     /* not supported on this device */
};

/* config flags */
#define XENG_NIBBLE_RE_LOW 0x1u   /* real part in the low nibble */
#define XENG_COUNTS 0x4u          /* keep per-pair sample counts (xeng_correlate_flagged, xeng_dump_counts) */

typedef struct {
    int32_t n_inputs;          /* 1 <= N <= 65535 receiver-polarizations per channel */
    int32_t n_slots;           /* independent accumulators (channels) >= 1 */
    int32_t device;            /* HIP device ordinal */
    uint32_t flags;            /* XENG_NIBBLE_RE_LOW or 0 */
    int64_t mem_budget_bytes;  /* cap on device bytes for accumulators; 0 = none */
} xeng_config;

/*
 * Create a correlator context (the channels a node serves, Sec. 2.3: each
 * slot integrates one channel's visibilities): allocates n_slots zeroed int32 accumulators
 * of xeng_slot_bytes(n_inputs) bytes each on `device`.  The library owns
 * them until xeng_destroy.  Returns XENG_EINVAL for bad fields,
 * XENG_ENOMEM if the accumulators exceed mem_budget_bytes or hipMalloc
 * fails, XENG_EDEVICE / XENG_ENOTSUP for device problems.
 */
int xeng_create(const xeng_config *cfg, xeng_ctx **out);

/* Free the context and its accumulators (synchronizes the device first). */
int xeng_destroy(xeng_ctx *ctx);

/*
 * Correlate n_samples time samples of one channel into slot `slot`
 * (Sec. 2.2, eta; the "Correlation" task of Table tab:computing):
 *   acc[slot] += V(d_samples[0 : n_samples])
 * d_samples: device pointer, time-major [n_samples][row_stride] bytes,
 *   owned by the caller.  n_samples >= 0 (0 is a no-op).
 *   N <= row_stride <= 2^26.
 * Asynchronous on hip_stream.  Refuses with XENG_EOVERFLOW if the slot
 * would integrate more than xeng_max_integration() samples.  On a slot
 * named by a live prepared batch (xeng_batch_create) the call first waits
 * for the device to read the slot's true count.
 * Samples whose base and row stride are multiples of 16 bytes with N a
 * multiple of 16 are read in place; otherwise, for N >= 256, the call first
 * copies them (in chunks of at most 256 MiB) into rows of N rounded up to
 * 16 bytes, in stream-ordered scratch from a pool the library keeps per
 * device (up to 1 GiB retained), and correlates the copy; XENG_ENOMEM if
 * that scratch cannot be had (nothing queued).  A device error in a later
 * chunk leaves the chunks already queued integrated and counted in
 * xeng_samples_integrated.
 */
int xeng_correlate(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples,
                   int64_t n_samples, int64_t row_stride, void *hip_stream);

/*
 * Allocation-free variant of xeng_correlate, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same result and the same checks, but nothing is
 * allocated, freed or pooled -- no cached plan, no padded copy.  The call's
 * work plan is written on the device, by a one-thread kernel queued ahead
 * of the correlation, into a fixed array of XENG_STATIC_SCRATCH_BYTES that
 * each GPU holds from the library's set-up until the process ends.  Every
 * call on a GPU shares that array (and each call overwrites it), so calls
 * that may overlap on one GPU -- on different streams, from different
 * threads -- race; calls ordered on one stream do not.  Samples the wide
 * kernel cannot read in place take the 128 x 128 kernel directly.
 * XENG_ENOMEM, nothing queued, if the plan would not fit the array (about
 * 65000 pieces: N = 2048 fits at any T up to xeng_max_integration()).
 * XENG_ENOTSUP while hip_stream is capturing, like xeng_correlate.
 */
#define XENG_STATIC_SCRATCH_BYTES (1 << 20)
int xeng_correlate_static(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples,
                          int64_t n_samples, int64_t row_stride, void *hip_stream);

/*
 * Flags and RFI excision (Sec. 2.2: every block of samples travels with
 * flags and metadata; Table tab:computing: an "RFI Excision" task runs on
 * the GPU ahead of the correlation).  A flag covers one input over a block
 * of block_len consecutive samples of a call (the last block may be
 * shorter): flags[b * N + i] != 0 means input i is flagged over samples
 * [b * block_len, (b + 1) * block_len).
 */
typedef struct {
    int32_t block_len;  /* samples per block, 2 .. XENG_RFI_MAX_BLOCK */
    int32_t den;        /* thresholds lo = lo_num / den, hi = hi_num / den; 1 <= den <= 1024 */
    int32_t lo_num;     /* 0 <= lo_num <= hi_num <= 16 * den */
    int32_t hi_num;
    int32_t reserved;   /* must be 0 */
} xeng_rfi_config;
#define XENG_RFI_MAX_BLOCK 1024

/*
 * RFI excision by spectral kurtosis (the estimator of Nita and Gary 2010;
 * the paper names the task, not the method): for each block of M samples
 * of each input, with P = |x|^2, S1 = sum P and S2 = sum P^2,
 *     SK = (M + 1) / (M - 1) * (M S2 / S1^2 - 1)
 * (expectation 1 for Gaussian noise; a steady carrier gives about 0,
 * impulsive interference much more than 1).  d_flags[b * N + i] = 1 where
 * SK < lo or SK > hi or S1 = 0, else 0; blocks of one sample are never
 * flagged.  The comparison is exact (integer arithmetic).  d_samples as in
 * xeng_correlate (N = n_inputs, `flags` = XENG_NIBBLE_RE_LOW or 0);
 * d_flags: device, ceil(n_samples / block_len) * N bytes, owned by the
 * caller.  Asynchronous on hip_stream; XENG_EINVAL for bad arguments (at
 * most 65535 blocks per call), XENG_ENOTSUP while capturing.
 */
int xeng_rfi_flags(const uint8_t *d_samples, int64_t n_samples, int32_t n_inputs, int64_t row_stride,
                   uint32_t flags, const xeng_rfi_config *cfg, uint8_t *d_flags, void *hip_stream);

/*
 * Flag-aware correlation into a context created with XENG_COUNTS:
 *   acc[slot]    += sum_t w_i(t) w_j(t) x_i(t) conj(x_j(t))
 *   counts[slot] += sum_t w_i(t) w_j(t)          (n_ij, per pair)
 * with w = 0 where the flag array marks the sample's (block, input), else
 * 1.  Flagged samples never enter a visibility; n_ij counts the samples
 * that did, so V_ij / n_ij is the mean over them.  The samples are copied
 * into padded rows with flagged samples set to zero (scratch from the
 * library's pool, in chunks as the padded path of xeng_correlate) and
 * correlated by the wide kernel.  Same checks and integration bound as
 * xeng_correlate; XENG_EINVAL without XENG_COUNTS or with block_len < 1.
 */
int xeng_correlate_flagged(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                           int64_t row_stride, const uint8_t *d_flags, int32_t block_len, void *hip_stream);

/*
 * Per-pair sample counts of a slot (XENG_COUNTS): out[k], int32
 * [N(N+1)/2] in the pair order of xeng_dump, = the samples integrated into
 * pair k since the slot's last reset (every sample of an unflagged call
 * counts for every pair).  Asynchronous; call it before the xeng_dump that
 * resets the slot (a reset clears the counts with the visibilities).
 */
int xeng_dump_counts(xeng_ctx *ctx, int32_t slot, int32_t *out, void *hip_stream);

/*
 * The same integration as xeng_correlate (same result, checks and bound),
 * computed in the paper's unsigned form (Sec. 2.3, "GPUs": low-bit
 * products at the cost of O(N) bookkeeping; Table tab:computing, "Re-Order
 * and Pre-Sum"): the matrix cores multiply the stored nibbles u = x + 8
 * (0..15) themselves, the pre-sums SR_i = sum_t uR_i and SI_i = sum_t uI_i
 * are added up per slot (by the wide kernel itself, else by a pass over
 * the samples), and a correction adds, per pair,
 *   Re: -8 (SR_i + SI_i + SR_j + SI_j) + 128 T,
 *   Im:  8 (SR_i - SI_i) - 8 (SR_j - SI_j).
 * The correction is linear in (SR, SI, T), so it is applied once for all
 * such calls on a slot, by the slot's next xeng_dump or xeng_dump_batch (on
 * that call's stream, which must be ordered after them, as for any dump),
 * or discarded by xeng_reset: a slot's exports are exactly those of
 * xeng_correlate.  A second, independent route to the same
 * integers on the GPU: the wide kernel's unsigned instance where the array
 * allows it in place (int8, or FP8 under XENG_KERNEL_FP8), else the
 * 128 x 128 kernel's (int8), which XENG_KERNEL_GENERAL also selects.  The
 * per-slot pre-sums (8 N bytes) are allocated with the context.
 */
int xeng_correlate_presum(xeng_ctx *ctx, int32_t slot, const uint8_t *d_samples, int64_t n_samples,
                          int64_t row_stride, void *hip_stream);

/*
 * Phased-array beamforming (Sec. 2.1: the nodes form 10 phased-array beams
 * for pulsar timing; "Pulsar Beamforming" in Table tab:computing):
 *     y_b(t) = sum_i w_bi x_i(t),   b < n_beams, t < n_samples,
 * with complex int8 weights, parts in [-127, 127].  A beam set holds the
 * weights on the device in the order the kernel's matrix-core operands read
 * them.  weights: HOST memory, int8 [n_beams][n_inputs][2] (re, im), read
 * before the call returns; XENG_EINVAL for a part equal to -128, for
 * n_beams outside 1..XENG_BEAMS_MAX, or for flags other than
 * XENG_NIBBLE_RE_LOW.  xeng_beams_create uploads synchronously;
 * xeng_beams_set_weights replaces the weights asynchronously on hip_stream
 * (beamform calls queued after it on that stream see the new weights; it
 * waits for the previous update's copy before reusing its pinned staging).
 */
#define XENG_BEAMS_MAX 16
typedef struct xeng_beams xeng_beams;
int xeng_beams_create(int32_t n_inputs, int32_t n_beams, int32_t device, uint32_t flags, const int8_t *weights,
                      xeng_beams **out);
int xeng_beams_set_weights(xeng_beams *bm, const int8_t *weights, void *hip_stream);
int xeng_beams_destroy(xeng_beams *bm);

/*
 * Form the beams of n_samples time samples: d_samples as in xeng_correlate
 * (N = the beam set's n_inputs).  shift = -1: d_out is int32
 * [n_samples][n_beams][2], the exact sums; shift = 0..24: d_out is int8
 * [n_samples][n_beams][2], each part divided by 2^shift, rounded half to
 * even and clipped to [-127, 127] (the 8 + 8-bit beam export: the paper's
 * 0.25 Gb/s of pulsar beams per node is 16 bits per beam sample).  Device
 * memory owned by the caller.  Asynchronous on hip_stream; XENG_ENOTSUP
 * while capturing.
 */
int xeng_beamform(xeng_beams *bm, const uint8_t *d_samples, int64_t n_samples, int64_t row_stride, int32_t shift,
                  void *d_out, void *hip_stream);

/* One unit of a batched correlation: correlate d_samples into ctx/slot. */
typedef struct {
    xeng_ctx *ctx;
    int32_t slot;
    int32_t reserved;          /* must be 0 */
    const uint8_t *d_samples;  /* device, [n_samples][row_stride] */
    int64_t n_samples;
    int64_t row_stride;
} xeng_job;

/*
 * Correlate many channels or sub-arrays, of uneven N and T, in one
 * persistent launch (the paper runs one channel per GPU, Sec. 2.3; this
 * call lets one GPU serve many).  Every result equals what xeng_correlate
 * would give for that job alone.  All contexts must be on one device; a
 * (ctx, slot) pair may appear at most once per batch.  Checks every job
 * before queuing anything.  Each call copies its job table and its plan
 * (recurring job sizes are planned once; the plans are kept on the host) to
 * the device on hip_stream through a pinned staging ring, and never
 * synchronizes the device, so that a loop of calls with changing sizes
 * keeps the GPU busy.  Jobs with N >= 256 that the wide kernel cannot read
 * in place (see xeng_correlate) are copied into padded rows in scratch from
 * the library's pool first, up to 256 MiB of them per call; the rest run
 * the 128 x 128 kernel.  For graph capture use xeng_batch_* below (which
 * reads every job in place).
 */
int xeng_correlate_batch(const xeng_job *jobs, int32_t n_jobs, void *hip_stream);

/*
 * Export the integrated visibilities of a slot (Sec. 2.1 / Sec. 3.1:
 * integrated visibilities are exported at a chosen cadence).
 * out: int32 [N(N+1)/2][2], device memory or host memory from
 *   hipHostMalloc; owned by the caller.  reset != 0 zeroes the slot and its
 *   sample counter after the export.  Asynchronous on hip_stream.  Exports
 *   of one slot must not run concurrently on different streams (they share
 *   the slot's diagonal staging, and a reset export writes the accumulators
 *   the other reads).  A slot integrated by xeng_correlate_presum (or an FP8
 *   call on the wide kernel) since its last export gets the pending O(N)
 *   correction (see xeng_correlate_presum) on hip_stream: inside the export
 *   when it resets, else into the accumulators first; xeng_dump_batch
 *   applies it per slot before its export, and xeng_reset discards it.
 */
int xeng_dump(xeng_ctx *ctx, int32_t slot, int32_t *out, int32_t reset, void *hip_stream);

typedef struct {
    xeng_ctx *ctx;
    int32_t slot;
    int32_t reset;             /* 0 or 1, as in xeng_dump */
    int32_t *out;              /* int32 [N(N+1)/2][2] of this ctx's N, as in xeng_dump */
    int32_t reserved;          /* must be 0 */
    int32_t pad;
} xeng_dump_job;

/*
 * Export many slots at once (the exports of Sec. 2.1 for every channel that
 * reaches its cadence together): each job's output equals what xeng_dump
 * would write for it, and reset jobs zero their slot and sample counter.
 * Two launches cover the whole batch (diagonal staging, then the export),
 * where one xeng_dump per slot runs each export as its own small launch.
 * All contexts must be on one device; a (ctx, slot) pair may appear at most
 * once; the outputs must not overlap one another or any accumulator.
 * Checks every job before queuing anything (XENG_EINVAL, nothing queued).
 * Asynchronous on hip_stream: the job table is copied to the device through
 * the same pinned staging ring as xeng_correlate_batch (the host waits only
 * when the launch that used a ring buffer eight calls earlier is still
 * running).  n_jobs == 0 is a no-op.
 */
int xeng_dump_batch(const xeng_dump_job *jobs, int32_t n_jobs, void *hip_stream);

/* Zero one slot's accumulators and sample counter (asynchronous). */
int xeng_reset(xeng_ctx *ctx, int32_t slot, void *hip_stream);

/* Samples integrated in a slot since its last reset (the integration length
 * the overflow bound of Sec. 2.2's 4+4-bit products limits); -1 on bad
 * arguments.  For a slot named by a live prepared batch the count lives on
 * the device: the call waits for the device and reads it. */
int64_t xeng_samples_integrated(const xeng_ctx *ctx, int32_t slot);

/* Largest number of samples a slot may integrate between resets. */
int64_t xeng_max_integration(void);

/* Device bytes of one slot for N inputs: its int32 accumulators plus the
 * staging the dump uses (admission control); -1 if N < 1.  A context
 * created with XENG_COUNTS holds 4 * N(N+1)/2 bytes more per slot. */
int64_t xeng_slot_bytes(int32_t n_inputs);

/* N and slot count of a context (-1 on NULL). */
int32_t xeng_n_inputs(const xeng_ctx *ctx);
int32_t xeng_n_slots(const xeng_ctx *ctx);

/* Human-readable text for a status code (static storage); the codes are
 * those of enum xeng_status above. */
const char *xeng_strerror(int status);

/*
 * Simple GPU reference correlator (one thread per pair, scalar int32 sums,
 * no MFMA, no tiling) writing the packed visibilities of one call straight
 * into d_out (overwritten, int32 [N(N+1)/2][2], device).  A debugging and
 * cross-checking path; n_samples <= xeng_max_integration().
 */
int xeng_correlate_reference(const uint8_t *d_samples, int64_t n_samples, int32_t n_inputs,
                             int64_t row_stride, uint32_t flags, int32_t *d_out,
                             void *hip_stream);

/*
 * Work decomposition (host only, no device needed).  The correlation of a
 * batch is split into pieces: a tile of the upper triangle of one job over
 * a contiguous range of samples, each piece run by one workgroup of the
 * persistent launch.  Tiles cut into several pieces are flushed with integer
 * atomic adds, the others with a plain add.  Jobs whose samples pointer and
 * row stride are multiples of 16 bytes and whose N is a multiple of 16 use
 * workgroup tiles of 128 x 256 inputs ("wide") -- or, for N <= 64, the
 * single 64 x 64 region of tile (0, 0) ("narrow": the workgroup's waves
 * split the piece's time) -- others 128 x 128.
 */
typedef struct {
    int32_t job;       /* index into the batch */
    int32_t ti, tj;    /* first accumulator tile: row / column in units of 128 inputs */
    int32_t atomic;    /* 1 if the tile is shared with other pieces */
    int64_t t0, t1;    /* sample range [t0, t1) */
    int32_t workgroup; /* workgroup that runs the piece */
    int32_t n_tiles;   /* accumulator tiles (ti, tj .. tj + n_tiles - 1) computed */
} xeng_piece_info;

/*
 * Fill `out` (capacity `cap`) with the pieces the library would launch for
 * jobs of sizes (n_inputs[k], n_samples[k]) on `n_workgroups` workgroups
 * with at least `min_stages` 64-sample stages per piece (0 = library
 * default), for square (wide = 0), wide (wide = 1) or narrow (wide = 2,
 * jobs of N <= 64 only) units.  Returns the
 * number of pieces (which may exceed cap: then only cap are written), or a
 * negative status.  A wide piece's tile below the diagonal or past N is
 * computed but not stored.
 */
int64_t xeng_plan_inspect(const int32_t *n_inputs, const int64_t *n_samples, int32_t n_jobs,
                          int32_t n_workgroups, int32_t min_stages, int32_t wide,
                          xeng_piece_info *out, int64_t cap);

/*
 * The pieces xeng_correlate_static would launch for one job of n_inputs x
 * n_samples on n_workgroups workgroups (host only; same conventions and
 * return value as xeng_plan_inspect, job index 0).  The static path's
 * device planner emits exactly these, and they equal xeng_plan_inspect's
 * for that single job.
 */
int64_t xeng_plan_inspect_static(int32_t n_inputs, int64_t n_samples, int32_t n_workgroups, int32_t min_stages,
                                 int32_t wide, xeng_piece_info *out, int64_t cap);

/*
 * Prepared batch, for repeated launches of the same jobs (a streaming loop,
 * a captured graph).  xeng_batch_create checks the jobs as
 * xeng_correlate_batch does, plans them, and copies the plan and the job
 * table into device memory that the batch owns (synchronously).  The jobs'
 * sample pointers are fixed: each launch reads whatever those buffers hold
 * when it runs.  The contexts must outlive the batch.
 *
 * xeng_batch_launch enqueues kernels only -- a one-thread guard kernel,
 * then one correlation launch per kernel kind (at most two); no copy, no
 * memset, no allocation -- so it may be captured into a hipGraph, and every
 * replay integrates again.  The integration bound is enforced on the
 * device: each slot named by a live batch keeps its sample counter in
 * device memory, and the guard kernel of every launch or replay advances
 * the counters of all the batch's slots only if none would pass
 * xeng_max_integration(); otherwise the launch integrates nothing at all
 * (counters and accumulators unchanged) and is counted as refused.
 * xeng_batch_check waits for the device and returns XENG_EOVERFLOW if any
 * launch or replay of the batch was refused since the previous check.
 * While a slot is named by a live batch, xeng_samples_integrated and the
 * calls that integrate into it wait for the device to read its counter,
 * and it is never treated as holding zeros.  xeng_batch_destroy (which
 * synchronizes the device) hands the count back to the host.
 */
typedef struct xeng_batch xeng_batch;
int xeng_batch_create(const xeng_job *jobs, int32_t n_jobs, xeng_batch **out);
int xeng_batch_launch(xeng_batch *b, void *hip_stream);
int xeng_batch_check(xeng_batch *b);
int xeng_batch_destroy(xeng_batch *b);

/* A launch configuration (xeng_autotune, xeng_tuning_lookup). */
typedef struct {
    int32_t kernel;        /* XENG_KERNEL_* */
    int32_t wgs_per_cu;    /* general kernel's workgroups per compute unit */
    int32_t min_stages;    /* minimum piece length, 64-sample stages */
    int32_t plan_order;    /* XENG_PLAN_* of single-job launches */
    double us_per_launch;  /* measured time of a tuned configuration, else 0 */
    int32_t source;        /* XENG_TUNE_SETTINGS, XENG_TUNE_MEASURED or XENG_TUNE_CACHE_FILE */
    int32_t saved;         /* xeng_autotune: 1 if the tune-cache file was written */
} xeng_tuning;

#define XENG_TUNE_SETTINGS 0    /* the global settings (xeng_set_tuning, xeng_set_plan_order) */
#define XENG_TUNE_MEASURED 1    /* chosen by xeng_autotune in this process */
#define XENG_TUNE_CACHE_FILE 2  /* read from the tune-cache file */

/*
 * Autotuner (Sec. 2.3: each GPU processes its share of frequency channels;
 * what runs fastest depends on their N and T).  Times every candidate launch
 * configuration on these jobs, `iters` launches each on hip_stream: the
 * kernel (the eight- or four-wave DMA kernel, or the general kernel with one
 * or two workgroups per CU), the minimum piece length and, for a single
 * job, the work order.  The trials read the jobs' samples and accumulate
 * into accumulators the library allocates for the call and frees after:
 * the jobs' slots, their contents and their sample counts are left as they
 * were.  The fastest configuration is kept for every later call on this
 * device whose jobs fall into the same class: the largest N, the
 * power-of-two classes of the largest T and of the number of jobs, and
 * whether any job can take the DMA kernel (so that a streaming server's
 * launches, whose job counts and lengths vary, find it).  The device's
 * tuned entries are then written to the tune-cache file of its
 * architecture (xeng_tune_cache_path), which the library reads when it
 * first uses a device in a later process; best->saved says whether that
 * write succeeded (a failed write is not an error).  Synchronous; refused
 * (XENG_ENOTSUP) while hip_stream is capturing.  Results never depend on
 * the configuration.  xeng_set_tuning discards every tuned entry of this
 * process (the file keeps them; a later xeng_autotune updates the file's
 * entry for its own class only).
 */
int xeng_autotune(const xeng_job *jobs, int32_t n_jobs, int32_t iters, void *hip_stream,
                  xeng_tuning *best);

/*
 * The configuration a batched call (or, for one job, xeng_correlate) of
 * these jobs would launch with now, and where it comes from (out->source).
 * Jobs as for xeng_correlate_batch; nothing is launched.
 */
int xeng_tuning_lookup(const xeng_job *jobs, int32_t n_jobs, xeng_tuning *out);

/*
 * Path of the tune-cache file for `device`'s architecture:
 * $XENG_TUNE_DIR/xeng_tune_<arch>.json, else under $XDG_CACHE_HOME/xeng,
 * else under $HOME/.cache/xeng.  The environment is read at every call; the
 * file itself is read once per process, when the library first uses the
 * device.  Writes at most len - 1 characters and a terminating zero into
 * buf (nothing if len is 0) and returns the path's full length;
 * XENG_ENOTSUP if none of the three variables is set, XENG_EDEVICE for a
 * device that does not exist.  The file holds one JSON object: the
 * architecture, and one entry per job class (N, T class, jobs class, DMA
 * eligibility) with the chosen kernel, workgroups per CU, minimum piece
 * length, work order and measured microseconds per launch.  Processes that
 * tune at the same time each write the whole file; the last write wins.
 */
int32_t xeng_tune_cache_path(int32_t device, char *buf, int32_t len);

/*
 * Streaming server (Sec. 2.1: every channel delivers a sample every 2.56 us
 * and its integrated visibilities are exported at a chosen cadence).
 * Channels of N inputs ingest frames of frame_len samples every
 * frame_period_us; the server keeps their accumulators on the device
 * (admitting channels as slots and device memory allow),
 * correlates every channel's newly arrived frames in one batched launch
 * about every launch_period_us (continuous batching: frames that arrive
 * while launches run join the next one), and exports each channel every
 * dump_frames frames into a device buffer of its own.
 */
typedef struct xeng_server xeng_server;

/*
 * Server flag: stagger the exports.  The channel in slot s is exported when
 * its frame count reaches m * dump_frames - phase(s), m = 1, 2, ..., with
 * phase(s) = s * dump_frames / max_channels (so its first export covers
 * fewer frames, every later one dump_frames).  The channels' exports then
 * spread over the export period instead of all falling in one launch.
 */
#define XENG_SERVER_STAGGER_EXPORTS 2u

typedef struct {
    int32_t n_inputs;         /* N of every channel */
    int32_t device;
    uint32_t flags;           /* XENG_NIBBLE_RE_LOW, XENG_SERVER_STAGGER_EXPORTS, or 0 */
    int32_t frame_len;        /* samples per frame (CHIME-shaped: 256) */
    int32_t dump_frames;      /* frames per export; frame_len * dump_frames <= xeng_max_integration() */
    int32_t ring_frames;      /* device ring of a host-sourced channel, in frames */
    int32_t max_inflight;     /* batched launches queued on the device at once, >= 1 */
    int32_t max_channels;     /* slots; 0 = as many as mem_budget_bytes holds */
    double frame_period_us;   /* frame cadence per channel (256 samples at 390625/s: 655.36) */
    double launch_period_us;  /* batching period */
    int64_t mem_budget_bytes; /* most device bytes for slots and rings (0 = no budget) */
    int32_t reserved;         /* must be 0 */
} xeng_server_config;

typedef struct {
    int64_t frames_released;  /* frames whose release time passed during the run */
    int64_t frames_done;      /* frames integrated */
    int64_t frames_dropped;   /* host-sourced frames lost to a full ingest ring */
    int64_t launches;
    int64_t dumps;
    int64_t backlog_frames;   /* released, not dropped, not yet integrated at the end */
    int64_t channels_waiting; /* admitted channels still waiting for a slot or memory at the end */
    int64_t device_bytes;     /* device memory the server holds for slots and rings */
    double seconds;           /* wall time of the run */
    double tcmacs;            /* integrated CMAC / wall time, 1e12/s */
    double p50_ms, p99_ms, max_ms;   /* frame latency: release -> its launch completed */
    double max_pass_ms;          /* the real-time loop's longest pass */
    double max_launch_call_ms;   /* the longest time to queue one launch and its exports */
    double max_copy_call_ms;     /* the longest time to queue one ingest copy or gather */
    int64_t frames_gathered;     /* host frames ingested by the gather kernel (the others by
                                    DMA-engine copies: sources not verified pinned and 16-byte aligned) */
} xeng_server_stats;

typedef struct {
    int32_t state;            /* 0 waiting for a slot, 1 streaming, 2 finished */
    int32_t slot;
    int64_t frames_done;
    int64_t dumps;
    int64_t last_dump_first_frame;   /* first frame of the last export, -1 if none */
    double admitted_s;        /* when it took its slot, seconds into the run; -1 if it has not */
} xeng_server_channel;

/*
 * Create a server; XENG_ENOMEM if not even one slot fits the budget.  No
 * device memory for channels is allocated here: a slot's accumulators and
 * export buffer (xeng_slot_bytes(N) + N(N+1)/2 * 8 bytes) are allocated
 * when a channel first takes it, a host source's ring (ring_frames *
 * frame_len * N bytes) when no finished host source left one; both stay
 * with the server for later channels and are freed by xeng_server_destroy.
 */
int xeng_server_create(const xeng_server_config *cfg, xeng_server **out);
int xeng_server_destroy(xeng_server *s);
/* Slots of the server: the most channels streaming at once (max_channels,
 * capped by how many slots mem_budget_bytes holds). */
int32_t xeng_server_max_channels(const xeng_server *s);
/*
 * Admit a channel.  Its frames come from `frames`, [n_frames][frame_len][N]
 * bytes, frame f being frames[f % n_frames]: device memory read in place, or
 * (host_frames = 1) pinned host memory copied into the channel's device
 * ring on release.  Caller-owned; must outlive the server.  Frame 0 is
 * released start_s seconds into the next run; total_frames frames (0 =
 * unlimited) are streamed.  The channel waits for admission, which the
 * run loop grants in order of arrival (no channel overtakes one that
 * waits): it needs a free slot and the device memory it lacks (the slot's
 * own at its first use, a ring for a host source unless a finished one left
 * one) within mem_budget_bytes and within the device's free memory at that
 * moment, less a 512 MiB reserve.  A slot freed by a finished channel keeps
 * its memory, so the next channel takes it at once.  Its stream starts
 * when it is admitted (frame 0 no earlier than start_s).
 */
int xeng_server_admit(xeng_server *s, const uint8_t *frames, int64_t n_frames, int32_t host_frames,
                      double start_s, int64_t total_frames, int32_t *channel);
/* Run the real-time loop for `seconds`, then wait for queued work; fills `stats`. */
int xeng_server_run(xeng_server *s, double seconds, xeng_server_stats *stats);
int xeng_server_channel_info(const xeng_server *s, int32_t channel, xeng_server_channel *info);
/*
 * Copy a channel's last export (int32 [N(N+1)/2][2], the frames
 * [last_dump_first_frame, + dump_frames)) to `out` (device or host memory,
 * synchronous).  XENG_EBUSY if its slot has since passed to another channel.
 */
int xeng_server_last_dump(xeng_server *s, int32_t channel, int32_t *out);

/*
 * Export ring of a channel (where its integrated visibilities go at every
 * export, Sec. 2.1: visibilities leave the node at a chosen cadence):
 * export k of the channel (k = 0, 1, ... in export order) is written to
 * ring + (k % n_entries) * N(N+1)/2 * 2 int32, in device memory or pinned
 * host memory, caller-owned, valid until the server is destroyed.  The
 * exports land in stream order; read them after xeng_server_run returns.
 * Without a ring (the default) each export goes to the slot's own buffer
 * and only the last is kept (xeng_server_last_dump).  Must be set before
 * the channel's first export (XENG_EBUSY after); ring NULL with
 * n_entries 0 sets none.  xeng_server_last_dump then reads the ring's
 * latest entry.
 */
int xeng_server_export_ring(xeng_server *s, int32_t channel, int32_t *ring, int32_t n_entries);

/* Kernel selection for xeng_set_tuning. */
#define XENG_KERNEL_AUTO 0     /* wide DMA kernel (eight waves) where the job allows it, else general */
#define XENG_KERNEL_GENERAL 1  /* always the general kernel */
#define XENG_KERNEL_DMA4 2     /* wide DMA kernel with four waves where the job allows it, else general */
/*
 * Exact FP8 products on v_mfma_f32_32x32x16_fp8_fp8 with fp32 sums kept
 * below 2^24, converted to int32 at the flush (Sec. 4.1: low-bit matrix
 * units as the way forward).  A single-channel xeng_correlate (and
 * xeng_correlate_presum) on an array the wide kernel reads in place runs
 * the unsigned form on the wide kernel's FP8 instance: a stored nibble u is
 * the E4M3 code of u * 2^-9 as it stands (subnormals and the first binade),
 * its negation the same code with the sign bit set; pieces of at most 582
 * stages; the O(N) pre-sum correction of xeng_correlate_presum.  Jobs of
 * xeng_correlate_batch that the wide kernel reads in place do the same
 * (their slots' pre-sums add up, the correction follows at the export).
 * Prepared batches (xeng_batch_*, whose replays the library does not see)
 * and other arrays take the general kernel's FP8 instance: each signed
 * 4-bit value as its E4M3 code, pieces below 2^17 samples.  The same
 * results as every other kernel.
 */
#define XENG_KERNEL_FP8 3

/*
 * Launch tuning: workgroups per compute unit of the general kernel (1 or 2),
 * the minimum piece length in 64-sample stages, and the kernel selection.
 * Values < 0 (or 0 for the first two) keep the current setting.  Applies to
 * later calls on every device and discards the autotuner's choices.  Results
 * never depend on these settings.
 */
int xeng_set_tuning(int32_t wgs_per_cu, int32_t min_stages, int32_t kernel);

/*
 * Work order of single-job launches (results never depend on it).
 * XENG_PLAN_XCD (the default): the job's tiles in Morton order, cut into
 * time segments of about the balanced share of a workgroup; the 32
 * workgroups that share one of MI355X's eight XCDs (and its L2) take
 * segments of one time window over a compact block of tiles, so that they
 * read the same input rows and columns at about the same time; the tiles'
 * tails go to the remaining workgroups.  XENG_PLAN_LINEAR: the stream-K
 * order (tiles in row order, each workgroup a contiguous range of (tile,
 * stage)).  Batches of several jobs and jobs too short for one 32-stage
 * segment per workgroup always take the linear order, as does
 * xeng_correlate_static.  Applies to later calls on every device and to
 * xeng_plan_inspect.
 */
#define XENG_PLAN_LINEAR 0
#define XENG_PLAN_XCD 1
int xeng_set_plan_order(int32_t order);

/*
 * Scratch of the padded path: the single-channel calls that copy their
 * samples into padded rows (see xeng_correlate) go in chunks of at most
 * `bytes` of scratch, and a batched call pads at most `bytes` of its jobs.
 * 0 restores the default (256 MiB).  Applies to later calls on every
 * device; results never depend on it (smaller chunks only mean more
 * launches).  XENG_EINVAL if bytes < 0.
 */
int xeng_set_pad_chunk_bytes(int64_t bytes);

/*
 * Clock probe, for measurement (results never depend on it).  `dev_buf` is
 * device memory on `device` of at least 4 int64, or NULL to stop.  While
 * set, every launch of the wide (DMA) correlation kernel on that device
 * stores, from its workgroup 0, the shader-clock cycle counter and the
 * 100 MHz real-time counter at the workgroup's start ([0], [1]) and end
 * ([2], [3]); the caller derives the shader clock the launch ran at as
 * ([2] - [0]) / (([3] - [1]) / 1e8).  The buffer stays the caller's and must
 * outlive the launches that write it.  XENG_EINVAL for a negative device,
 * XENG_EDEVICE if the device cannot be set up.
 */
int xeng_clock_probe(int32_t device, int64_t *dev_buf);

/*
 * Matrix-core ceiling, for measurement (Table tab:computing puts three
 * quarters of the node's time in the correlation; this bounds how fast any
 * int8 kernel can run it here).  Runs, synchronously on `device`'s null
 * stream for about `ms` milliseconds, a loop of nothing but
 * v_mfma_i32_32x32x32_i8 on every compute unit in the wide correlation
 * kernel's shape (eight waves per CU, eight 32 x 32 accumulators per wave)
 * on operands of the correlator's form that change every instruction, and
 * stores the int8 MAC/s of the second half (the first lets the clock
 * settle under the load) and the shader clock of that half, in GHz.  The
 * chip's power limit holds its clock below the 2.4 GHz its peak is quoted
 * at under such a load, and the rate follows.  Allocates (device memory,
 * events) and waits for the device.  XENG_EINVAL for a negative device, ms
 * outside 10..10000 or null outputs; XENG_EDEVICE, XENG_ENOMEM on HIP
 * failures.
 */
int xeng_mfma_ceiling(int32_t device, int32_t ms, double *mac_per_s, double *sclk_ghz);

#ifdef __cplusplus
}
#endif

#endif /* XENG_H */
