// Internal layout constants and structures shared by the host runtime and
// the gfx950 kernels.  Nothing here is part of the public ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace xeng {

// ---------------------------------------------------------------------------
// Tiling.  The upper triangle of the N x N visibility matrix (Sec. 2.2: the
// N(N+1)/2 pairs including autocorrelations) is covered by TILE x TILE tiles
// (ti <= tj).  A tile is computed by one workgroup as 4 x 4 MFMA blocks of
// 32 x 32.
// ---------------------------------------------------------------------------
constexpr int TILE = 128;          // inputs per tile side
constexpr int BLK = 32;            // MFMA block side
constexpr int BLKS = TILE / BLK;   // 4 blocks per tile side
constexpr int STAGE = 64;          // samples per pipeline stage (LDS buffer)
constexpr int KSTEP = 16;          // samples per MFMA k-step (32 int8 values)

// Accumulator layout of one slot (device): tile-major over the upper
// triangle of tiles, tile index ti*nt - ti*(ti-1)/2 + (tj-ti).  Inside a
// tile: [ca][cb][reg][lane] of 64-bit words, with ca, cb the 4 x 4 blocks
// and (reg, lane) the MFMA 32 x 32 accumulator register layout: row r of the
// tile is in block ca = r / 32, column c in block cb = c / 32, and within a
// block row i, column j sit in register 4*(i/8) + i%4 of lane
// j + 32*((i/4)%2).  A word holds the pair (Re, Im) as Im * 2^32 + Re (Re
// sign-extended): 64-bit addition of such words adds both parts at once
// (one atomic per pair), and since each true sum fits in int32, Re is the
// low half read as int32 and Im = (word - Re) >> 32.
constexpr int64_t TILE_I32 = (int64_t)BLKS * BLKS * 2 * 16 * 64;   // 32768 int32 = 16384 words
constexpr int64_t BLOCK_I32 = 2 * 16 * 64;                          // 2048 int32 = 1024 words
constexpr int64_t TILE_W = TILE_I32 / 2;
constexpr int64_t BLOCK_W = BLOCK_I32 / 2;

__host__ __device__ inline uint64_t pack_pair(int32_t re, int32_t im)
{
    return ((uint64_t)(uint32_t)im << 32) + (uint64_t)(int64_t)re;
}
__host__ __device__ inline int32_t pair_re(uint64_t w) { return (int32_t)(uint32_t)w; }
__host__ __device__ inline int32_t pair_im(uint64_t w)
{
    return (int32_t)(uint32_t)((w - (uint64_t)(int64_t)pair_re(w)) >> 32);
}

inline int64_t tri64(int64_t n) { return n * (n + 1) / 2; }
__host__ __device__ inline int n_tiles_side_hd(int n) { return (n + TILE - 1) / TILE; }
inline int n_tiles_side(int n) { return (n + TILE - 1) / TILE; }
inline int64_t slot_i32(int n) { return tri64(n_tiles_side(n)) * TILE_I32; }
// Per-slot staging of the diagonal's imaginary parts for the dump.
inline int64_t diag_i32(int n) { return ((int64_t)n + 63) / 64 * 64; }

// Register sums of one piece: the general kernel's B operands carry 16x the
// sample values, so its sums reach 16 * 128 * length (pieces below 2^20
// samples); the DMA kernel's A and B both do, 256 * 128 * length (pieces
// below 2^16 samples).
constexpr int MAX_PIECE_STAGES = ((1 << 20) - 1) / STAGE;       // 16383 stages
constexpr int MAX_PIECE_STAGES_WIDE = ((1 << 16) - 1) / STAGE;  // 1023 stages
// The general kernel on unsigned nibbles: at most 8 x 450 per sample, so
// pieces below 2^19 samples keep the sums in int32.
constexpr int MAX_PIECE_STAGES_UNSIGNED = ((1 << 19) - 1) / STAGE;   // 8191 stages
// The wide kernel's FP8 products of unsigned nibbles: fp32 sums of at most
// 450 per sample stay exact integers below 2^24 over 582 stages.
constexpr int MAX_PIECE_STAGES_FP8_UNSIGNED = ((1 << 24) - 1) / (450 * STAGE);   // 582 stages

// Largest row stride: lane offsets inside a stage (up to 31 rows) stay 32-bit.
// Most workgroups one tile is shared among in a launch.  Every share of a
// tile flushes all of it with atomics, and shares of one tile end together,
// so their atomics meet on the same addresses: past about 16 shares the
// flush costs more than the extra workgroups save (measured on N = 64 to
// 512 with T of 4096 and 8192).
constexpr int64_t MAX_UNIT_SPLIT = 16;

constexpr int64_t MAX_STRIDE = INT64_C(1) << 26;

// Largest number of samples a slot may integrate: the largest |term| of
// x_i conj(x_j) with parts in [-8, 7] is 128 (Re), so 128 * T_MAX <= 2^31-1.
constexpr int64_t T_MAX = (INT64_C(2147483647)) / 128;   // 16,777,215

// Job descriptor read by the kernels (one per channel / sub-array).
struct JobDesc {
    const uint8_t *samples;   // [T][stride]
    int32_t *acc;             // slot accumulator base
    int64_t stride;           // bytes between time samples
    int32_t n;                // inputs
    int32_t nt;               // tiles per side
    uint32_t flags;           // JOB_* bits
    int32_t pad;
    int32_t *presum;          // optional: the slot's pre-sums ([SR | SI], N rounded up to 4 apart) for the
                              // wide kernel's FP8 instance of the unsigned form in a batch
};
constexpr uint32_t JOB_RE_LOW = 1u;    // real part in the low nibble
constexpr uint32_t JOB_ALIGNED8 = 2u;   // samples, stride and N are multiples of 8 bytes
constexpr uint32_t JOB_DMA = 4u;        // samples and stride multiples of 16 bytes, N of 16: DMA kernel
constexpr uint32_t JOB_FRESH = 8u;      // the slot holds zeros: whole-tile flushes store instead of add

// Work decomposition shapes: 128 x 128 tiles (general kernel), 128 x 256
// workgroup tiles covering two accumulator tiles (DMA kernel), or a narrow
// job's single 64 x 64 region (narrow kernel, N <= NARROW_MAX_N).
enum class TileShape { Square = 0, Wide = 1, Narrow = 2 };
constexpr int NARROW_MAX_N = 64;
constexpr int NARROW_WGS_PER_CU = 2;   // the narrow kernel's workgroups resident per CU

// One piece of work: tile (ti, tj) of job `job` over samples [t0, t1).
struct Piece {
    int32_t job;
    int32_t tile;       // ti | tj << 16
    int32_t t0;
    int32_t t1_atomic;  // t1 | (atomic << 31)
};

struct KernelArgs {
    JobDesc job0;             // used when jobs == nullptr (single job)
    const JobDesc *jobs;
    const Piece *pieces;
    const int32_t *wg_off;    // pieces of workgroup w: [wg_off[w], wg_off[w+1])
    const uint8_t *zeros;     // ZERO_BYTES bytes of zero samples (0x88), 16-byte aligned
    int64_t *clock;           // optional (DMA kernel): workgroup 0 stores {shader cycles, 100 MHz time} at start and end
    const int32_t *skip;      // optional: nonzero at launch time -> the launch integrates nothing
    int32_t *presum;          // optional (the wide kernel's unsigned instances): SR, SI (n4 = N rounded
                              // up to 4 apart) of the job's inputs, added to atomically
};

// Device-side integration guard of a prepared batch: one entry per job,
// the slot's device sample counter and the samples one launch adds.
struct GuardJob {
    int64_t *count;
    int64_t n;
};
constexpr int ZERO_BYTES = 256;

// One export of a batched dump: a slot's accumulators, its diagonal staging
// (n int32) and the caller's output, [n(n+1)/2][2] int32.
struct DumpDesc {
    int32_t *acc;
    int32_t *diag;
    int32_t *out;
    int32_t n;
    int32_t nt;
    int32_t reset;
    int32_t pad;
};

}  // namespace xeng
