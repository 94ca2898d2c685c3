// gfx950 correlation kernel for narrow jobs: N <= 64 inputs (a multiple of
// 16) with 16-byte-aligned sample arrays.
//
// The product is the wide DMA kernel's -- for the upper triangle,
//   V_ij = sum_t x_i(t) conj(x_j(t))                      (Sec. 2.2, eta)
// on v_mfma_i32_32x32x32_i8, with the same operand forms (B = [16 R | 16 I],
// A = [16 R | 16 I] for the real part and [16 I | 16 ~R] for the imaginary
// one, so the stored imaginary part is Im V_ij - S_j) and the same slot
// layout -- but the work is split the other way.  At N <= 64 the whole
// triangle is one 64 x 64 region (MFMA blocks (0,0), (0,1), (1,1) of one
// tile) and there are only 130 MACs per input byte: the wide kernel's
// eight waves would leave seven idle.  Here the four waves of a workgroup
// split a piece's time instead: wave w takes stages w, w + 4, ... and
// accumulates the whole region over them; the four partial sums are added
// into LDS by LDS atomics, and the four waves then flush a quarter of the
// region each (the read-modify-write of a slot in flight from every wave at
// once, not from one).  Two workgroups share a CU (two waves per SIMD), so
// one's loads, LDS round trips and unpack overlap the other's MFMAs, and
// one's reduction and flush at the end of a piece overlap the other's
// streaming.
//
//   * global -> registers: a stage (64 time rows x 64 inputs, 4 KiB) is four
//     16-byte loads per lane, three stages ahead of their use, so that every
//     CU keeps 96 KiB in flight.  Every load is issued, whatever the stage: rows at
//     or past the piece's end read the zero-sample buffer instead, so the
//     count of loads in flight is the same at every point of the loop and
//     the waits for a stage's data wait for that stage only;
//   * registers -> LDS in the wide kernel's chunk-major layout (chunk c of
//     row r at byte 128 c + 16 r of its 8-row group), in a buffer private to
//     the wave: the main loop needs no barrier;
//   * LDS -> registers by transposed reads (ds_read_b64_tr_b8); since rows
//     and columns are the same 64 inputs, each read is both an A and a B
//     operand (the B operand is the real form of the A block of the same
//     inputs).
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {
namespace narrow {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) v2i lds_v2i;
typedef __attribute__((address_space(1))) uint64_t gw64;
typedef __attribute__((address_space(1))) const v4i gv4i;

constexpr int WAVES = 4;
constexpr int WIDTH = 64;                      // inputs of a stage row
constexpr int STAGE_BYTES = STAGE * WIDTH;     // 4 KiB
constexpr int GROUP = 8 * WIDTH;               // an 8-row group: 512 bytes
constexpr int BLOCKS = 3;                      // (0,0), (0,1), (1,1)
constexpr int PARTIAL_I32 = BLOCKS * 2 * 16;   // accumulator registers per lane
// LDS: a stage buffer per wave, then the workgroup's sums of a piece
// ([PARTIAL_I32][64] int32, 24 KiB): 56 KiB, within the 64 KiB a workgroup
// may declare statically
constexpr int SUM_OFFSET = WAVES * STAGE_BYTES;
constexpr int LDS_BYTES = SUM_OFFSET + PARTIAL_I32 * 64 * 4;
// (block, register) rows of the sums each wave flushes
constexpr int ROWS_PER_WAVE = BLOCKS * 16 / WAVES;
static_assert(BLOCKS * 16 % WAVES == 0, "the sums split evenly over the waves");

__device__ __forceinline__ constexpr int blk_a(int k) { return k == 2 ? 1 : 0; }
__device__ __forceinline__ constexpr int blk_b(int k) { return k == 0 ? 0 : 1; }

struct Acc {
    v16i re[BLOCKS];
    v16i im[BLOCKS];
};

// A wave-uniform 64-bit value moved to scalar registers (the job and piece
// fields come from memory, so the compiler cannot tell they are uniform;
// in scalar registers every branch and loop bound on them is scalar too,
// and the waits for loads in flight stay exact).
template <typename T> __device__ __forceinline__ T uniform(T v)
{
    static_assert(sizeof(T) == 8, "64-bit values only");
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    u = ((uint64_t)hi << 32) | lo;
    __builtin_memcpy(&v, &u, 8);
    return v;
}

// One stage of this lane: rows 16 k + lane / 4, inputs 16 (lane % 4) .. + 15
// (the last 16 inputs for a chunk at or past n: what they add reaches only
// pairs with i or j >= n, which are never exported).  Rows at or past t1
// read 16 bytes of the zero-sample buffer.
struct StageRegs {
    v4i d[4];
};

__device__ __forceinline__ void load_stage(StageRegs &g, const JobDesc &jd, const uint8_t *zeros, int t, int t1,
                                           int lane)
{
    const int c = lane & 3, r = lane >> 2;
    const int in = min(16 * c, jd.n - 16);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int row = t + 16 * k + r;
        const uint8_t *src = row < t1 ? jd.samples + (int64_t)row * jd.stride + in : zeros + 16 * (lane & 15);
        g.d[k] = *(gv4i *)src;
    }
}

__device__ __forceinline__ void store_stage(uint8_t *buf, const StageRegs &g, int lane)
{
    const int c = lane & 3, r = lane >> 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int row = 16 * k + r;   // group row / 8, row % 8 within it
        *reinterpret_cast<v4i *>(buf + (row >> 3) * GROUP + 128 * c + 16 * (row & 7)) = g.d[k];
    }
}

// Unpacked operands of one 32-input block for one k-step: {16R, 16R, 16I,
// 16I, 16~R, 16~R} (real A = elements 0..3, which is also the B form;
// imaginary A = elements 2..5).
__device__ __forceinline__ v8i unpack(v2i raw, bool re_low)
{
    const uint32_t x0 = (uint32_t)raw.x, x1 = (uint32_t)raw.y;
    const uint32_t s0 = x0 << 4, s1 = x1 << 4;
    const uint32_t h0 = (x0 ^ 0x88888888u) & 0xF0F0F0F0u, h1 = (x1 ^ 0x88888888u) & 0xF0F0F0F0u;
    const uint32_t l0 = (s0 ^ 0x80808080u) & 0xF0F0F0F0u, l1 = (s1 ^ 0x80808080u) & 0xF0F0F0F0u;
    if (re_low) {
        const uint32_t n0 = (s0 ^ 0x70707070u) & 0xF0F0F0F0u, n1 = (s1 ^ 0x70707070u) & 0xF0F0F0F0u;
        return v8i{(int)l0, (int)l1, (int)h0, (int)h1, (int)n0, (int)n1, 0, 0};
    }
    const uint32_t n0 = (x0 ^ 0x77777777u) & 0xF0F0F0F0u, n1 = (x1 ^ 0x77777777u) & 0xF0F0F0F0u;
    return v8i{(int)h0, (int)h1, (int)l0, (int)l1, (int)n0, (int)n1, 0, 0};
}

// The four k-steps (16 samples each) of one stage in the wave's buffer:
// the transposed reads of k-step q + 1 are issued before the unpack and
// the MFMAs of k-step q, so the LDS round trip hides behind them.  TWO:
// N > 32, so blocks (0,1) and (1,1) hold pairs of the triangle (else only
// block (0,0) is computed).
template <bool RE_LOW, bool TWO>
__device__ __forceinline__ void stage_mfma(Acc &acc, const uint8_t *buf, int lane)
{
    constexpr int NA = TWO ? 2 : 1;   // 32-input blocks read per k-step
    const int grp = lane >> 4, jl = lane & 15;
    // group 2q + grp / 2 (time rows 16 q.., this lane's half of the k-step),
    // chunk 2 a + grp % 2 (inputs 32 a + 16 (grp % 2)..), byte 8 jl
    uint8_t *base = const_cast<uint8_t *>(buf) + GROUP * (grp >> 1) + 128 * (grp & 1) + 8 * jl;
    // an explicit cast of a pointer into the workgroup's shared array to
    // the LDS address space
    auto read = [&](int q, int a) {
        return __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(base + 2 * GROUP * q + 256 * a));
    };
    v2i raw[2][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) raw[0][a] = read(0, a);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < 3)
#pragma unroll
            for (int a = 0; a < NA; ++a) raw[(q + 1) & 1][a] = read(q + 1, a);
        v8i o[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) o[a] = unpack(raw[q & 1][a], RE_LOW);
#pragma unroll
        for (int k = 0; k < (TWO ? BLOCKS : 1); ++k) {
            const v4i re_a = __builtin_shufflevector(o[blk_a(k)], o[blk_a(k)], 0, 1, 2, 3);
            const v4i b = __builtin_shufflevector(o[blk_b(k)], o[blk_b(k)], 0, 1, 2, 3);
            acc.re[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a, b, acc.re[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < (TWO ? BLOCKS : 1); ++k) {
            const v4i im_a = __builtin_shufflevector(o[blk_a(k)], o[blk_a(k)], 2, 3, 4, 5);
            const v4i b = __builtin_shufflevector(o[blk_b(k)], o[blk_b(k)], 0, 1, 2, 3);
            acc.im[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a, b, acc.im[k], 0, 0, 0);
        }
    }
}

// This wave's stages of a piece: its k-th is stage wave + 4 k.  Four
// register stages rotate with fixed roles in a loop unrolled by four: the
// loads of stage k + 3 are issued as stage k is used, so three stages are in
// flight behind the one in use (stages past the wave's last read zero
// samples and are never used), and no register stage is copied (a copy
// would wait for the newest loads).
template <bool RE_LOW, bool TWO>
__device__ __forceinline__ void run_piece(Acc &acc, uint8_t *buf, const JobDesc &jd, const uint8_t *zeros, int t0,
                                          int t1, int wave, int lane)
{
    const int ns = (t1 - t0 + STAGE - 1) / STAGE;
    const int m = wave < ns ? (ns - wave + WAVES - 1) / WAVES : 0;   // this wave's stages
    auto t_of = [&](int k) { return t0 + STAGE * (wave + WAVES * k); };
    auto use = [&](const StageRegs &g) {
        store_stage(buf, g, lane);
        stage_mfma<RE_LOW, TWO>(acc, buf, lane);
    };
    StageRegs g0, g1, g2, g3;
    load_stage(g0, jd, zeros, t_of(0), t1, lane);
    load_stage(g1, jd, zeros, t_of(1), t1, lane);
    load_stage(g2, jd, zeros, t_of(2), t1, lane);
    int k = 0;
    for (; k + 4 <= m; k += 4) {
        load_stage(g3, jd, zeros, t_of(k + 3), t1, lane);
        use(g0);
        load_stage(g0, jd, zeros, t_of(k + 4), t1, lane);
        use(g1);
        load_stage(g1, jd, zeros, t_of(k + 5), t1, lane);
        use(g2);
        load_stage(g2, jd, zeros, t_of(k + 6), t1, lane);
        use(g3);
    }
    if (k < m) use(g0);
    if (k + 1 < m) use(g1);
    if (k + 2 < m) use(g2);
}

// This wave's (block, register) rows of the workgroup's sums to the slot:
// rows wave * ROWS_PER_WAVE .., row 16 k + r being register r of block k
// for every lane (64 pairs).  The old values of a read-modify-write are all
// loaded before any is stored back.
__device__ __forceinline__ void flush_rows(const JobDesc &jd, const int32_t *sum, bool atomic, int wave, int lane)
{
    gw64 *w[ROWS_PER_WAVE];
    uint64_t v[ROWS_PER_WAVE];
#pragma unroll
    for (int i = 0; i < ROWS_PER_WAVE; ++i) {
        const int row = wave * ROWS_PER_WAVE + i, k = row / 16, r = row % 16;
        w[i] = (gw64 *)jd.acc + (blk_a(k) * BLKS + blk_b(k)) * BLOCK_W + r * 64 + lane;   // tile (0, 0)
        v[i] = pack_pair(sum[((2 * k) * 16 + r) * 64 + lane] >> 8, sum[((2 * k + 1) * 16 + r) * 64 + lane] >> 8);
    }
    if (atomic) {
#pragma unroll
        for (int i = 0; i < ROWS_PER_WAVE; ++i)
            __hip_atomic_fetch_add(w[i], v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    uint64_t old[ROWS_PER_WAVE];
    const bool fresh = (jd.flags & JOB_FRESH) != 0;
#pragma unroll
    for (int i = 0; i < ROWS_PER_WAVE; ++i) old[i] = fresh ? 0 : *w[i];
#pragma unroll
    for (int i = 0; i < ROWS_PER_WAVE; ++i) *w[i] = old[i] + v[i];
}

// A wave's partial sums into the workgroup's, [register row][lane] int32,
// by LDS atomic adds.
__device__ __forceinline__ void add_to_sum(int32_t *sum, const Acc &acc, int lane)
{
#pragma unroll
    for (int k = 0; k < BLOCKS; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            atomicAdd(&sum[((2 * k) * 16 + r) * 64 + lane], acc.re[k][r]);
            atomicAdd(&sum[((2 * k + 1) * 16 + r) * 64 + lane], acc.im[k][r]);
        }
}

// Persistent kernel: workgroup w runs pieces [wg_off[w], wg_off[w+1]), each
// a time range [t0, t1) of one narrow job's single unit.
__global__ __launch_bounds__(64 * WAVES) void xcorr_narrow(KernelArgs args)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    // a prepared batch's device guard refused this launch
    if (args.skip != nullptr && *args.skip != 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint8_t *buf = lds + wave * STAGE_BYTES;
    int32_t *sum = reinterpret_cast<int32_t *>(lds + SUM_OFFSET);
    const int p_begin = args.wg_off[blockIdx.x], p_end = args.wg_off[blockIdx.x + 1];
    for (int pi = p_begin; pi < p_end; ++pi) {
        const Piece pce = args.pieces[pi];
        JobDesc jd = args.jobs ? args.jobs[__builtin_amdgcn_readfirstlane(pce.job)] : args.job0;
        jd.samples = uniform(jd.samples);
        jd.acc = uniform(jd.acc);
        jd.stride = uniform(jd.stride);
        jd.n = __builtin_amdgcn_readfirstlane(jd.n);
        jd.flags = (uint32_t)__builtin_amdgcn_readfirstlane((int)jd.flags);
        const int t1a = __builtin_amdgcn_readfirstlane(pce.t1_atomic);
        const bool atomic = t1a < 0;
        const int t0 = __builtin_amdgcn_readfirstlane(pce.t0), t1 = t1a & 0x7FFFFFFF;
        // the workgroup's sums start at zero (the previous piece's flush
        // has read them: the barrier at the end of its loop iteration)
        for (int i = threadIdx.x; i < PARTIAL_I32 * 64 / 4; i += 64 * WAVES)
            reinterpret_cast<v4i *>(sum)[i] = v4i{0, 0, 0, 0};
        Acc acc;
#pragma unroll
        for (int k = 0; k < BLOCKS; ++k)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc.re[k][r] = 0;
                acc.im[k][r] = 0;
            }
        const bool re_low = (jd.flags & JOB_RE_LOW) != 0, two = jd.n > 32;
        if (re_low && two)
            run_piece<true, true>(acc, buf, jd, args.zeros, t0, t1, wave, lane);
        else if (re_low)
            run_piece<true, false>(acc, buf, jd, args.zeros, t0, t1, wave, lane);
        else if (two)
            run_piece<false, true>(acc, buf, jd, args.zeros, t0, t1, wave, lane);
        else
            run_piece<false, false>(acc, buf, jd, args.zeros, t0, t1, wave, lane);
        __syncthreads();   // the sums are zeroed
        add_to_sum(sum, acc, lane);
        __syncthreads();   // every wave's partial sums are in
        flush_rows(jd, sum, atomic, wave, lane);
        __syncthreads();   // the flush has read the sums
    }
}

}  // namespace narrow

hipError_t launch_correlate_narrow(const KernelArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(narrow::xcorr_narrow, dim3(grid), dim3(64 * narrow::WAVES), 0, stream, a);
    return hipGetLastError();
}

}  // namespace xeng
