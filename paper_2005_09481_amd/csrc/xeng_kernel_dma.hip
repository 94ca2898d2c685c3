// gfx950 correlation kernel for 16-byte-aligned sample arrays of N a
// multiple of 256.
//
// Same product as the general kernel -- for a tile of the upper triangle,
//   V_ij = sum_t x_i(t) conj(x_j(t))                      (Sec. 2.2, eta)
// with Re V = [Re x_i | Im x_i] . [Re x_j | Im x_j] and
//      Im V = [Im x_i | -Re x_i] . [Re x_j | Im x_j]
// on v_mfma_i32_32x32x32_i8 -- but the packed samples never leave their
// 4-bit form in shared memory:
//   * global -> LDS by DMA (global_load_lds_dwordx4): 16 bytes per lane, no
//     registers and no instructions beyond the load itself, into a ring of
//     NSLOT 64-sample stages so that NSLOT - 1 stages are in flight;
//   * LDS -> registers by transposed reads (ds_read_b64_tr_b8): a 16-lane
//     group reads 8 time rows x 16 inputs and each lane receives the 8
//     samples of one input -- exactly one lane's share of an MFMA operand;
//   * the nibble unpack to int8 happens in registers right before the MFMA.
// The LDS bytes per MFMA are a quarter of an unpacked layout's.
//
// Workgroup tile: 128 rows (A) x 256 columns (B), four waves; wave (wa, wb)
// computes rows 64wa..64wa+63 against columns 128wb..128wb+127, i.e. 2 x 4
// MFMA blocks for both Re and Im (256 accumulator registers).
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {
namespace dma {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) v2i lds_v2i;
typedef __attribute__((address_space(1))) int32_t gi32;

constexpr int WA_ROWS = 128;            // A rows per workgroup tile
constexpr int WB_COLS = 256;            // B columns per workgroup tile
constexpr int CA = WA_ROWS / 16;        // 16-input chunks per A time row (8)
constexpr int CB = WB_COLS / 16;        // 16
constexpr int A_STAGE = STAGE * WA_ROWS;    // 8 KB of packed samples
constexpr int B_STAGE = STAGE * WB_COLS;    // 16 KB
constexpr int SLOT = A_STAGE + B_STAGE;     // 24 KB
constexpr int NSLOT = 6;                    // ring depth: 144 KB of LDS
constexpr int DEPTH = NSLOT - 1;            // stages in flight
constexpr int DMA_A = A_STAGE / 1024;       // 1 KB DMA instructions per stage: 8
constexpr int DMA_B = B_STAGE / 1024;       // 16
constexpr int DMA_PER_WAVE = (DMA_A + DMA_B) / 4;   // 6

// Swizzled position of 16-byte chunk c of time row t in a region with C
// chunks per row: the 8 rows a transposed read touches land in 8 different
// bank groups.
__device__ __forceinline__ int chunk_index(int t, int c, int C) { return t * C + (c ^ (t & 7)); }

// s_waitcnt immediates: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and
// lgkmcnt 11:8 at their maxima (no wait on those).
#define XENG_VMCNT(n) (((n) & 0xF) | (((n) >> 4) << 14) | (0x7 << 4) | (0xF << 8))

struct Tile {
    const uint8_t *samples;
    int64_t stride;
    int n;
    int row0, col0;       // first A input, first B input
    int t0, t1;
};

// One 16-byte-per-lane DMA from global memory (uniform base + 32-bit lane
// offset) into LDS at byte offset `lds_base` + 16 * lane.  Written as
// inline assembly so that the compiler, which cannot tell that reads of
// other ring slots never alias the slot being filled, does not drain every
// load in flight before each LDS read; the ring's own vmcnt waits
// order the accesses.  The instruction has no register result; M0 (its LDS
// base) is saved and restored around it.
__device__ __forceinline__ void dma16(const uint8_t *base, uint32_t lane_off, uint32_t lds_base)
{
    // both are wave-uniform; readfirstlane puts them in scalar registers (its
    // result is a signed int: widen each half as unsigned)
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint32_t b_hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint32_t b_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint64_t sb = ((uint64_t)b_hi << 32) | (uint64_t)b_lo;
    const uint32_t sl = (uint32_t)__builtin_amdgcn_readfirstlane(lds_base);
    uint32_t saved;
    // s_nop 4: the LDS DMA may read M0 only one wait state after an SALU
    // write to it, and an SGPR address only five after a VALU write
    asm volatile("s_mov_b32 %0, m0\n\t"
                 "s_mov_b32 m0, %3\n\t"
                 "s_nop 4\n\t"
                 "global_load_lds_dwordx4 %1, %2\n\t"
                 "s_mov_b32 m0, %0"
                 : "=&s"(saved)
                 : "v"(lane_off), "s"(sb), "s"(sl)
                 : "memory");
}

// Lane geometry of this wave's k-th DMA instruction of a stage: time row in
// the stage and input byte offset in a row (inputs at or past N are
// redirected to input 0; their samples are masked at unpack).
__device__ __forceinline__ void dma_lane(const Tile &tl, int wave, int lane, int k, int &t, uint32_t &col)
{
    const int inst = wave + 4 * k;
    const bool in_a = inst < DMA_A;
    const int C = in_a ? CA : CB;
    const int first = in_a ? inst * 64 : (inst - DMA_A) * 64;
    const int ci = first + lane;
    t = ci / C;
    const int c = (ci % C) ^ (t & 7);
    const int in0 = (in_a ? tl.row0 : tl.col0) + 16 * c;
    col = (uint32_t)(in0 < tl.n ? in0 : 0);
}

// Per-lane byte offsets (row * stride + input) of this wave's six DMA
// instructions from a stage's first row, fixed for a piece.
struct DmaLane {
    uint32_t off[DMA_PER_WAVE];
};

__device__ __forceinline__ void dma_lane_setup(DmaLane &dl, const Tile &tl, int wave, int lane)
{
#pragma unroll
    for (int k = 0; k < DMA_PER_WAVE; ++k) {
        int t;
        uint32_t col;
        dma_lane(tl, wave, lane, k, t, col);
        dl.off[k] = (uint32_t)(t * tl.stride) + col;
    }
}

// This wave's share of one stage's DMA: instructions wave, wave+4, ... of the
// 24 (8 for A, 16 for B).  Rows at or past t1 (the last, partial stage of a
// piece, and the dummy stages past its end that keep the count of loads in
// flight constant) are redirected to the piece's first row.
__device__ __forceinline__ void issue_dma(uint32_t slot_lds, const Tile &tl, const DmaLane &dl, int stage,
                                          int wave, int lane)
{
    const int ts = tl.t0 + stage * STAGE;
    if (ts + STAGE <= tl.t1) {
        const uint8_t *row0 = tl.samples + (int64_t)ts * tl.stride;
#pragma unroll
        for (int k = 0; k < DMA_PER_WAVE; ++k) {
            const int inst = wave + 4 * k;
            const bool in_a = inst < DMA_A;
            const int first = in_a ? inst * 64 : (inst - DMA_A) * 64;
            dma16(row0, dl.off[k], slot_lds + (in_a ? 0 : A_STAGE) + 16 * first);
        }
    } else {
        const uint8_t *row0 = tl.samples + (int64_t)tl.t0 * tl.stride;
#pragma unroll
        for (int k = 0; k < DMA_PER_WAVE; ++k) {
            const int inst = wave + 4 * k;
            const bool in_a = inst < DMA_A;
            const int first = in_a ? inst * 64 : (inst - DMA_A) * 64;
            int t;
            uint32_t col;
            dma_lane(tl, wave, lane, k, t, col);
            const uint32_t off = ts + t < tl.t1 ? (uint32_t)((ts - tl.t0 + t) * tl.stride) + col : col;
            dma16(row0, off, slot_lds + (in_a ? 0 : A_STAGE) + 16 * first);
        }
    }
}

// Transposed read of one MFMA operand's packed samples: the lane gets the 8
// samples (k-step q, half lane / 32) of input 16 * chunk + lane % 32, as laid
// out by issue_dma.  `region` is an LDS byte offset.
__device__ __forceinline__ v2i read_tr(uint32_t region, int C, int q, int chunk, int lane)
{
    const int grp = lane >> 4, j = lane & 15;
    const int c = chunk + (grp & 1);
    const int t = 16 * q + 8 * (grp >> 1) + (j >> 1);
    const uint32_t off = region + 16 * chunk_index(t, c, C) + 8 * (j & 1);
    return __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(uintptr_t)off);
}

__device__ __forceinline__ uint32_t nib_to_i8(uint32_t n) { return (n + 0x78787878u) ^ 0x80808080u; }
__device__ __forceinline__ uint32_t nib_to_neg_i8(uint32_t n) { return (0x88888888u - n) ^ 0x80808080u; }

// A operands: Re-A = [Re | Im], Im-A = [Im | -Re] (int8).
template <bool RE_LOW>
__device__ __forceinline__ void unpack_a(v2i p, v4i &re_a, v4i &im_a)
{
    const uint32_t h0 = ((uint32_t)p.x >> 4) & 0x0F0F0F0Fu, l0 = (uint32_t)p.x & 0x0F0F0F0Fu;
    const uint32_t h1 = ((uint32_t)p.y >> 4) & 0x0F0F0F0Fu, l1 = (uint32_t)p.y & 0x0F0F0F0Fu;
    const uint32_t r0 = RE_LOW ? l0 : h0, i0 = RE_LOW ? h0 : l0;
    const uint32_t r1 = RE_LOW ? l1 : h1, i1 = RE_LOW ? h1 : l1;
    const uint32_t re0 = nib_to_i8(r0), re1 = nib_to_i8(r1);
    const uint32_t im0 = nib_to_i8(i0), im1 = nib_to_i8(i1);
    re_a = v4i{(int)re0, (int)re1, (int)im0, (int)im1};
    im_a = v4i{(int)im0, (int)im1, (int)nib_to_neg_i8(r0), (int)nib_to_neg_i8(r1)};
}

// B operand: [16 Re | 16 Im] (flipping bit 3 of an offset-binary nibble gives
// its 4-bit two's complement; in the high half of a byte that is 16x).
template <bool RE_LOW>
__device__ __forceinline__ v4i unpack_b(v2i p)
{
    const uint32_t x0 = (uint32_t)p.x ^ 0x88888888u, x1 = (uint32_t)p.y ^ 0x88888888u;
    const uint32_t h0 = x0 & 0xF0F0F0F0u, l0 = (x0 << 4) & 0xF0F0F0F0u;
    const uint32_t h1 = x1 & 0xF0F0F0F0u, l1 = (x1 << 4) & 0xF0F0F0F0u;
    return RE_LOW ? v4i{(int)l0, (int)l1, (int)h0, (int)h1} : v4i{(int)h0, (int)h1, (int)l0, (int)l1};
}

// Replace samples past t1 by the zero sample 0x88: `keep` holds the byte
// masks of the lane's 8 samples.
__device__ __forceinline__ v2i mask_samples(v2i p, uint32_t keep_lo, uint32_t keep_hi)
{
    return v2i{(int)(((uint32_t)p.x & keep_lo) | (0x88888888u & ~keep_lo)),
               (int)(((uint32_t)p.y & keep_hi) | (0x88888888u & ~keep_hi))};
}

// Byte mask of the first `n` (clamped to 0..4) bytes of a dword.
__device__ __forceinline__ uint32_t byte_mask(int n)
{
    return n >= 4 ? 0xFFFFFFFFu : n <= 0 ? 0u : (1u << (8 * n)) - 1u;
}

struct Acc {
    v16i re[2][4];
    v16i im[2][4];
};

// Packed operand data of one k-step: 2 A blocks and 4 B blocks.
struct Raw {
    v2i a[2];
    v2i b[4];
};

__device__ __forceinline__ void read_kstep(Raw &r, uint32_t slot, int q, int lane, int wa, int wb)
{
#pragma unroll
    for (int a = 0; a < 2; ++a) r.a[a] = read_tr(slot, CA, q, 4 * wa + 2 * a, lane);
#pragma unroll
    for (int b = 0; b < 4; ++b) r.b[b] = read_tr(slot + A_STAGE, CB, q, 8 * wb + 2 * b, lane);
}

// The 64 MFMAs of one stage for wave (wa, wb) from ring slot `slot`.  The
// packed operands of k-step q+1 are read while those of k-step q are
// unpacked and multiplied.  EDGE: the stage has samples past t1, which are
// masked to zero samples.
template <bool RE_LOW, bool EDGE>
__device__ __forceinline__ void stage_compute(Acc &acc, uint32_t slot, const Tile &tl, int ts,
                                              int lane, int wa, int wb)
{
    Raw raw;
    read_kstep(raw, slot, 0, lane, wa, wb);
#pragma unroll
    for (int q = 0; q < STAGE / KSTEP; ++q) {
        Raw cur = raw;
        if (q + 1 < STAGE / KSTEP) read_kstep(raw, slot, q + 1, lane, wa, wb);
        if (EDGE) {
            const int nt = tl.t1 - (ts + 16 * q + 8 * (lane >> 5));
            const uint32_t lo = byte_mask(nt), hi = byte_mask(nt - 4);
#pragma unroll
            for (int a = 0; a < 2; ++a) cur.a[a] = mask_samples(cur.a[a], lo, hi);
#pragma unroll
            for (int b = 0; b < 4; ++b) cur.b[b] = mask_samples(cur.b[b], lo, hi);
        }
        v4i re_a[2], im_a[2], bo[4];
#pragma unroll
        for (int a = 0; a < 2; ++a) unpack_a<RE_LOW>(cur.a[a], re_a[a], im_a[a]);
#pragma unroll
        for (int b = 0; b < 4; ++b) bo[b] = unpack_b<RE_LOW>(cur.b[b]);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                acc.re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a[a], bo[b], acc.re[a][b], 0, 0, 0);
                acc.im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a[a], bo[b], acc.im[a][b], 0, 0, 0);
            }
    }
}

// Accumulators hold 16x the visibilities (B operands are scaled by 16), so
// the flush adds acc >> 4; every value is a multiple of 16, so this is exact.
__device__ __forceinline__ void flush_block(int32_t *blk_, const v16i &re, const v16i &im, bool atomic)
{
    gi32 *blk = (gi32 *)blk_;
    if (atomic) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            __hip_atomic_fetch_add(blk + r * 64, re[r] >> 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(blk + 1024 + r * 64, im[r] >> 4, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            blk[r * 64] += re[r] >> 4;
            blk[1024 + r * 64] += im[r] >> 4;
        }
    }
}

// One piece: full stages in a single-path loop (the accumulators stay in
// place), then the partial last stage, if any, with masking.  Every stage
// slot gets exactly DMA_PER_WAVE loads per wave, so one constant wait
// (4 newer stages in flight) makes stage s complete.
template <bool RE_LOW>
__device__ __forceinline__ void run_piece(Acc &acc, uint32_t ring, const Tile &tl, int wave, int lane,
                                          int wa, int wb)
{
    const int len = tl.t1 - tl.t0;
    const int nfull = len / STAGE;
    DmaLane dl;
    dma_lane_setup(dl, tl, wave, lane);
    // nothing else in flight: the ring's vmcnt waits then count DMA only
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) issue_dma(ring + d * SLOT, tl, dl, d, wave, lane);
    int s = 0;
    for (; s < nfull; ++s) {
        __builtin_amdgcn_s_waitcnt(XENG_VMCNT((DEPTH - 1) * DMA_PER_WAVE));
        __syncthreads();   // stage s complete in LDS; stage s-1 no longer read
        issue_dma(ring + ((s + DEPTH) % NSLOT) * SLOT, tl, dl, s + DEPTH, wave, lane);
        stage_compute<RE_LOW, false>(acc, ring + (s % NSLOT) * SLOT, tl, tl.t0 + s * STAGE, lane, wa, wb);
    }
    if (nfull * STAGE < len) {
        __builtin_amdgcn_s_waitcnt(XENG_VMCNT((DEPTH - 1) * DMA_PER_WAVE));
        __syncthreads();
        stage_compute<RE_LOW, true>(acc, ring + (s % NSLOT) * SLOT, tl, tl.t0 + s * STAGE, lane, wa, wb);
    }
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
    __syncthreads();       // the next piece's DMA reuses the slots
}

// Persistent kernel: workgroup w runs pieces [wg_off[w], wg_off[w+1]).  A
// piece's tile field holds (I, J2): A rows 128 I.., B columns 256 J2.., i.e.
// accumulator tiles (I, 2 J2) and (I, 2 J2 + 1) where they are in the upper
// triangle.
__global__ __launch_bounds__(256, 1) void xcorr_dma(KernelArgs args)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    // LDS byte address of the ring, wave-uniform (scalar register)
    const uint32_t ring = (uint32_t)__builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wb = wave & 1;

    const int p_begin = args.wg_off[blockIdx.x], p_end = args.wg_off[blockIdx.x + 1];
    for (int pi = p_begin; pi < p_end; ++pi) {
        const Piece pce = args.pieces[pi];
        const JobDesc jd = args.jobs ? args.jobs[pce.job] : args.job0;
        const int ti = pce.tile & 0xFFFF, tj2 = (pce.tile >> 16) & 0xFFFF;
        const bool atomic = pce.t1_atomic < 0;
        Tile tl;
        tl.samples = jd.samples;
        tl.stride = jd.stride;
        tl.n = jd.n;
        tl.row0 = ti * WA_ROWS;
        tl.col0 = tj2 * WB_COLS;
        tl.t0 = pce.t0;
        tl.t1 = pce.t1_atomic & 0x7FFFFFFF;
        // this wave's accumulator tile; a half below the diagonal or past N
        // is computed (the workgroup stays in step) but not stored
        const int tj = 2 * tj2 + wb;
        const bool valid = tj >= ti && tj < jd.nt;

        Acc acc;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc.re[a][b][r] = 0;
                    acc.im[a][b][r] = 0;
                }
        if (jd.flags & JOB_RE_LOW)
            run_piece<true>(acc, ring, tl, wave, lane, wa, wb);
        else
            run_piece<false>(acc, ring, tl, wave, lane, wa, wb);

        if (valid) {
            const int64_t tile_idx = (int64_t)ti * jd.nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
            int32_t *tb = jd.acc + tile_idx * TILE_I32 + lane;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    flush_block(tb + ((2 * wa + a) * BLKS + b) * BLOCK_I32, acc.re[a][b], acc.im[a][b],
                                atomic);
                    // one block at a time: keeps the register file for the main loop
                    __builtin_amdgcn_sched_barrier(0);
                }
        }
    }
}

}  // namespace dma

constexpr int DMA_LDS_BYTES = dma::NSLOT * dma::SLOT;

hipError_t launch_correlate_dma(const KernelArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)dma::xcorr_dma,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, DMA_LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(dma::xcorr_dma, dim3(grid), dim3(256), DMA_LDS_BYTES, stream, a);
    return hipGetLastError();
}

}  // namespace xeng
