// gfx950 correlation kernel for 16-byte-aligned sample arrays (base and row
// stride) of N a multiple of 16.
//
// Same product as the general kernel -- for a tile of the upper triangle,
//   V_ij = sum_t x_i(t) conj(x_j(t))                      (Sec. 2.2, eta)
// on v_mfma_i32_32x32x32_i8 -- but the packed samples never leave their
// 4-bit form in shared memory:
//   * global -> LDS by DMA (global_load_lds_dwordx4): 16 bytes per lane, no
//     registers and no instructions beyond the load itself, into a ring of
//     NSLOT 64-sample stages, AHEAD of them issued before they are needed;
//   * LDS -> registers by transposed reads (ds_read_b64_tr_b8): a 16-lane
//     group reads 8 time rows x 16 inputs and each lane receives the 8
//     samples of one input -- exactly one lane's share of an MFMA operand;
//   * the nibble unpack to int8 happens in registers, one k-step ahead of
//     the MFMAs that use it.
//
// Operands.  With R, I the 4-bit parts of a sample (two's complement values
// in [-8, 7]) and ~R = -R - 1:
//   B (columns j)      = [16 R_j | 16 I_j]
//   A, real part       = [16 R_i | 16 I_i]   -> 256 (R_i R_j + I_i I_j)
//   A, imaginary part  = [16 I_i | 16 ~R_i]  -> 256 (I_i R_j - R_i I_j - I_j)
// Every byte is a 4-bit value in the high half of a byte, made from the
// packed sample by one XOR and one AND (no sign extension), and ~R never
// overflows int8 where -R would (R = -8).  The imaginary accumulator thus
// holds Im V_ij - S_j with S_j = sum_t I_j(t); since Im V_jj = 0 its diagonal
// holds -S_j, and the dump subtracts it.  The general kernel stores the same
// form.
//
// Workgroup tile: 128 rows (A) x 256 columns (B), NW waves in two rows of
// NW / 2; wave (wa, wb) computes rows 64wa..64wa+63 against 256 / (NW / 2)
// columns, i.e. 2 x BW MFMA blocks for both Re and Im.  Four waves (one per
// SIMD, 256 accumulator registers each) read the fewest operand bytes per
// MFMA; eight (two per SIMD, 128 each; the default) let one wave's MFMAs run
// while the other waits on LDS, a barrier or its DMA issue -- with eight,
// waves 0..3 (one per SIMD) issue all of a stage's DMA, since a burst of DMA
// instructions holds the issuing wave for tens of cycles per instruction.
// Regions and blocks wholly below the diagonal are not computed.
//
// LDS stage layout ("chunk-major" in 8-row groups): the A region holds 8
// groups of 8 time rows x 8 chunks of 16 inputs, chunk c of row r at byte
// 128 c + 16 r of its group; the B region the same with 16 chunks.  The 8
// rows a transposed read touches are then 128 contiguous bytes, and every
// read of a stage is a per-lane base plus a compile-time offset.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {
namespace dma {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) v2i lds_v2i;
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(1))) uint64_t gw64;

constexpr int WA_ROWS = 128;            // A rows per workgroup tile
constexpr int WB_COLS = 256;            // B columns per workgroup tile
constexpr int GRP_A = 8 * WA_ROWS;      // bytes of an 8-row group, A region: 1 KB
constexpr int GRP_B = 8 * WB_COLS;      // 2 KB
constexpr int A_STAGE = STAGE * WA_ROWS;    // 8 KB of packed samples
constexpr int B_STAGE = STAGE * WB_COLS;    // 16 KB
constexpr int SLOT = A_STAGE + B_STAGE;     // 24 KB
constexpr int NSLOT = 6;                    // ring: 144 KB of LDS
constexpr int AHEAD = NSLOT - 1;            // stages issued ahead
constexpr int DMA_A = A_STAGE / 1024;       // 1 KB DMA instructions per stage: 8
constexpr int DMA_B = B_STAGE / 1024;       // 16

// With eight waves, the DMA is left to one wave per SIMD (the other wave's
// MFMAs then run while the issuing wave waits to issue); 0 spreads it over
// all eight.
#ifndef XENG_DMA_SPLIT
#define XENG_DMA_SPLIT 1
#endif

template <int NW> struct Layout {
    static constexpr int WB_WAVES = NW / 2;                  // waves across the 256 columns
    static constexpr int BW = 8 / WB_WAVES;                  // B blocks per wave
    static constexpr int DMA_WAVES = (NW == 8 && XENG_DMA_SPLIT) ? 4 : NW;   // waves that issue DMA
    static constexpr int DMA_PER_WAVE = (DMA_A + DMA_B) / DMA_WAVES;
    static constexpr int MFMA_PER_K = 4 * BW;                // MFMAs per k-step
    static constexpr int READS_PER_K = 2 + BW;               // transposed reads per k-step
    static constexpr int VALU_PER_MFMA = NW == 4 ? 3 : 4;    // unpack share between MFMAs
};

// s_waitcnt immediates: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and
// lgkmcnt 11:8 at their maxima (no wait on those); and lgkmcnt(0) alone.
#define XENG_VMCNT(n) (((n) & 0xF) | (((n) >> 4) << 14) | (0x7 << 4) | (0xF << 8))
#define XENG_LGKMCNT0 (0xF | (0x3 << 14) | (0x7 << 4))

// A wave-uniform 64-bit value moved to scalar registers.
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

struct Tile {
    const uint8_t *samples;
    const uint8_t *zeros;   // 16 bytes of zero samples (0x88)
    int64_t stride;
    int n;                  // inputs (a multiple of 16)
    int row0, col0;         // first A input, first B input
    int t0, t1;
};

// 16-byte-per-lane DMAs into LDS at byte address `lds_addr` + 16 * lane,
// written as inline assembly so that the compiler, which cannot tell that
// reads of other ring slots never alias the slot being filled, does not
// drain every load in flight before each LDS read; the ring's own vmcnt
// waits order the accesses.  The instructions have no register result; M0
// (their LDS base) is saved and restored around them.  Wait states: one
// between an SALU write of M0 and the DMA; five between a VALU write of an
// SGPR (readfirstlane) and a memory instruction that reads it as its base.
// (readfirstlane is a no-op on values already in scalar registers; it
// returns a signed int, so each half of a pointer is widened as unsigned.)
//
// Vector-address form: a 64-bit address per lane.
__device__ __forceinline__ void dma16_v(const uint8_t *addr, uint32_t lds_addr)
{
    const uint32_t sl = (uint32_t)__builtin_amdgcn_readfirstlane(lds_addr);
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\t"
                 "s_mov_b32 m0, %2\n\t"
                 "s_nop 0\n\t"
                 "global_load_lds_dwordx4 %1, off\n\t"
                 "s_mov_b32 m0, %0"
                 : "=&s"(saved)
                 : "v"(addr), "s"(sl)
                 : "memory");
}

// Scalar-base form, wave-uniform 64-bit base + per-lane 32-bit offsets: a
// whole stage's share of DMAs (K = 6 or 3) in one statement:
// M0 saved once, one s_nop 4 ahead of the first instruction (covering a
// VALU write of any SGPR operand, which the statement's own instructions
// never make), and between instructions only the one wait state an SALU
// write of M0 needs before an LDS DMA.
template <int K>
__device__ __forceinline__ void dma16_s_stage(const uint8_t *base, const uint32_t (&lane_off)[K],
                                              const uint32_t (&lds_addr)[K])
{
    static_assert(K == 6 || K == 3, "6 or 3 instructions per wave");
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint32_t b_hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint32_t b_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint64_t sb = ((uint64_t)b_hi << 32) | (uint64_t)b_lo;
    uint32_t sl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sl[k] = (uint32_t)__builtin_amdgcn_readfirstlane(lds_addr[k]);
    uint32_t saved;
    if constexpr (K == 6) {
        asm volatile("s_mov_b32 %0, m0\n\t"
                     "s_mov_b32 m0, %8\n\t"
                     "s_nop 4\n\t"
                     "global_load_lds_dwordx4 %1, %7\n\t"
                     "s_mov_b32 m0, %9\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %2, %7\n\t"
                     "s_mov_b32 m0, %10\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %3, %7\n\t"
                     "s_mov_b32 m0, %11\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %4, %7\n\t"
                     "s_mov_b32 m0, %12\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %5, %7\n\t"
                     "s_mov_b32 m0, %13\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %6, %7\n\t"
                     "s_mov_b32 m0, %0"
                     : "=&s"(saved)
                     : "v"(lane_off[0]), "v"(lane_off[1]), "v"(lane_off[2]), "v"(lane_off[3]),
                       "v"(lane_off[4]), "v"(lane_off[5]), "s"(sb), "s"(sl[0]), "s"(sl[1]), "s"(sl[2]),
                       "s"(sl[3]), "s"(sl[4]), "s"(sl[5])
                     : "memory");
    } else {
        asm volatile("s_mov_b32 %0, m0\n\t"
                     "s_mov_b32 m0, %5\n\t"
                     "s_nop 4\n\t"
                     "global_load_lds_dwordx4 %1, %4\n\t"
                     "s_mov_b32 m0, %6\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %2, %4\n\t"
                     "s_mov_b32 m0, %7\n\t"
                     "s_nop 0\n\t"
                     "global_load_lds_dwordx4 %3, %4\n\t"
                     "s_mov_b32 m0, %0"
                     : "=&s"(saved)
                     : "v"(lane_off[0]), "v"(lane_off[1]), "v"(lane_off[2]), "s"(sb), "s"(sl[0]), "s"(sl[1]),
                       "s"(sl[2])
                     : "memory");
    }
}

// Geometry of DMA instruction `inst` (0..23) of a stage for this lane: its
// LDS offset in the slot (wave-uniform), the time row in the stage and the
// first of the 16 inputs the lane fetches.  Instructions 0..7 fill A group
// `inst`; 8..23 fill half h of B group g.  Lane l fetches chunk l / 8 of
// the instruction's 8 chunks at time row l % 8 of the group, which lands at
// byte 16 l = 128 (l / 8) + 16 (l % 8) of the instruction's kilobyte.
// A chunk at or past input n (the edge tiles of an N that is not a multiple
// of the tile) is fetched from inputs n - 16.. instead: every load stays in
// its row, and what lands in those rows or columns of the tile only reaches
// accumulator entries (i, j) with i or j >= n, which are never exported.
__device__ __forceinline__ void dma_geom(int inst, int lane, int n, int row0, int col0, int &lds_off, int &t,
                                         int &in)
{
    const int r = lane & 7, c = lane >> 3;
    if (inst < DMA_A) {
        lds_off = inst * GRP_A;
        t = 8 * inst + r;
        in = row0 + 16 * c;
    } else {
        const int i = inst - DMA_A, g = i >> 1, h = i & 1;
        lds_off = A_STAGE + g * GRP_B + h * 1024;
        t = 8 * g + r;
        in = col0 + 16 * (8 * h + c);
    }
    in = min(in, n - 16);
}

// Index of this wave among the DMA-issuing waves, or -1.  Waves 0..3 sit on
// SIMDs 0..3 (waves of a workgroup are placed on the SIMDs in turn).
template <int NW> __device__ __forceinline__ int dma_wave(int wave)
{
    if (Layout<NW>::DMA_WAVES == NW) return wave;
    return wave < 4 ? wave : -1;
}

// Per-lane byte offsets (row * stride + input) of this wave's DMA
// instructions from a stage's first row, fixed for a piece.
template <int NW> struct DmaLane {
    uint32_t off[Layout<NW>::DMA_PER_WAVE];
};

template <int NW>
__device__ __forceinline__ void dma_lane_setup(DmaLane<NW> &dl, const Tile &tl, int wave, int lane)
{
#pragma unroll
    for (int k = 0; k < Layout<NW>::DMA_PER_WAVE; ++k) {
        int lds_off, t, in;
        dma_geom(dma_wave<NW>(wave) + Layout<NW>::DMA_WAVES * k, lane, tl.n, tl.row0, tl.col0, lds_off, t, in);
        dl.off[k] = (uint32_t)((int64_t)t * tl.stride) + (uint32_t)in;
    }
}

// This wave's share of one stage's DMA: instructions dw, dw + DMA_WAVES, ...
// of the 24, dw being the wave's index among the issuing waves (the others
// issue none).  Rows at or past t1 (the last, partial stage of a piece, and stages
// past its end, issued so that the count of loads in flight stays
// constant) are read from the zero-sample buffer, so that every stage the
// compute loop sees is whole.
template <int NW>
__device__ __forceinline__ void issue_stage(uint32_t slot_addr, const Tile &tl, const DmaLane<NW> &dl, int stage,
                                            int wave, int lane)
{
    const int dw = dma_wave<NW>(wave);
    if (dw < 0) return;
    const int ts = tl.t0 + stage * STAGE;
    if (ts + STAGE <= tl.t1) {
        const uint8_t *row = tl.samples + (int64_t)ts * tl.stride;
        uint32_t lds[Layout<NW>::DMA_PER_WAVE];
#pragma unroll
        for (int k = 0; k < Layout<NW>::DMA_PER_WAVE; ++k) {
            int lds_off, t, in;
            dma_geom(dw + Layout<NW>::DMA_WAVES * k, lane, tl.n, tl.row0, tl.col0, lds_off, t, in);
            lds[k] = slot_addr + (uint32_t)lds_off;
        }
        dma16_s_stage<Layout<NW>::DMA_PER_WAVE>(row, dl.off, lds);
    } else {
#pragma unroll
        for (int k = 0; k < Layout<NW>::DMA_PER_WAVE; ++k) {
            int lds_off, t, in;
            dma_geom(dw + Layout<NW>::DMA_WAVES * k, lane, tl.n, tl.row0, tl.col0, lds_off, t, in);
            const uint8_t *src =
                ts + t < tl.t1 ? tl.samples + (int64_t)(ts + t) * tl.stride + in : tl.zeros;
            dma16_v(src, slot_addr + (uint32_t)lds_off);
        }
    }
}

// Packed operand data of one k-step (2 A blocks, BW B blocks) and its
// unpacked form.
template <int NW> struct Raw {
    v2i a[2];
    v2i b[Layout<NW>::BW];
};
template <int NW> struct Ops {
    v8i a[2];   // {16R, 16R, 16I, 16I, 16~R, 16~R, -, -}: real A = s0123, imaginary A = s2345
    v4i b[Layout<NW>::BW];   // {16R, 16R, 16I, 16I}
};
template <int NW, bool F> struct Acc {
    v16i re[2][Layout<NW>::BW];
    v16i im[2][Layout<NW>::BW];
};
template <int NW> struct Acc<NW, true> {
    v16f re[2][Layout<NW>::BW];
    v16f im[2][Layout<NW>::BW];
};

// Transposed reads of k-step q: `pa`, `pb` are this lane's bases in the
// slot's A and B regions (group lane / 32, chunk of the lane's 16-lane
// group, byte 8 (lane % 16)); k-step q adds 2 groups, block a / b 2 chunks.
template <int NW>
__device__ __forceinline__ void read_k(Raw<NW> &r, const lds_u8 *pa, const lds_u8 *pb, int q)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
        r.a[a] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(pa + 2 * GRP_A * q + 256 * a));
#pragma unroll
    for (int b = 0; b < Layout<NW>::BW; ++b)
        r.b[b] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(pb + 2 * GRP_B * q + 256 * b));
}

// 16 x (4-bit value) in the high half of each byte: from the high nibbles,
// (p ^ 0x88) & 0xF0 per byte; from the low nibbles, the same on p << 4.
// XOR with 0x77 instead of 0x88 gives 16 x the bitwise complement.
//
// Unsigned form (U): the stored nibbles u in 0..15 themselves, no offset
// removed -- A real [uR | uI], A imaginary [uI | -uR] (per byte
// (0x80 - u) ^ 0x80: no borrows), B [8 uR | 8 uI] (at most 120) -- so the
// sums are 8 x the exact products of the stored values, with no bias.
//
// FP8 form (F, unsigned): a byte holding u in 0..15 is the OCP E4M3 code of
// u x 2^-9 (codes 0..7 are the subnormals m x 2^-9, codes 8..15 the first
// binade (8 + m) x 2^-9), and setting its top bit negates it exactly.  So A
// real [uR | uI], A imaginary [uI | -uR] and B [uR | uI] are the masked
// nibbles themselves (and the sign bit), and the fp32 sums hold the exact
// integer sums x 2^-18.
template <int NW, bool RE_LOW, bool U, bool F>
__device__ __forceinline__ void unpack_k(Ops<NW> &o, const Raw<NW> &r)
{
    if constexpr (F) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const uint32_t x0 = (uint32_t)r.a[a].x, x1 = (uint32_t)r.a[a].y;
            const uint32_t h0 = (x0 >> 4) & 0x0F0F0F0Fu, h1 = (x1 >> 4) & 0x0F0F0F0Fu;
            const uint32_t l0 = x0 & 0x0F0F0F0Fu, l1 = x1 & 0x0F0F0F0Fu;
            const uint32_t re0 = RE_LOW ? l0 : h0, re1 = RE_LOW ? l1 : h1;
            const uint32_t im0 = RE_LOW ? h0 : l0, im1 = RE_LOW ? h1 : l1;
            o.a[a] = v8i{(int)re0, (int)re1, (int)im0, (int)im1, (int)(re0 | 0x80808080u), (int)(re1 | 0x80808080u),
                         0, 0};
        }
#pragma unroll
        for (int b = 0; b < Layout<NW>::BW; ++b) {
            const uint32_t x0 = (uint32_t)r.b[b].x, x1 = (uint32_t)r.b[b].y;
            const uint32_t h0 = (x0 >> 4) & 0x0F0F0F0Fu, h1 = (x1 >> 4) & 0x0F0F0F0Fu;
            const uint32_t l0 = x0 & 0x0F0F0F0Fu, l1 = x1 & 0x0F0F0F0Fu;
            o.b[b] = RE_LOW ? v4i{(int)l0, (int)l1, (int)h0, (int)h1} : v4i{(int)h0, (int)h1, (int)l0, (int)l1};
        }
        return;
    }
    if constexpr (U) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const uint32_t x0 = (uint32_t)r.a[a].x, x1 = (uint32_t)r.a[a].y;
            const uint32_t h0 = (x0 >> 4) & 0x0F0F0F0Fu, h1 = (x1 >> 4) & 0x0F0F0F0Fu;
            const uint32_t l0 = x0 & 0x0F0F0F0Fu, l1 = x1 & 0x0F0F0F0Fu;
            const uint32_t re0 = RE_LOW ? l0 : h0, re1 = RE_LOW ? l1 : h1;
            const uint32_t im0 = RE_LOW ? h0 : l0, im1 = RE_LOW ? h1 : l1;
            const uint32_t n0 = (0x80808080u - re0) ^ 0x80808080u, n1 = (0x80808080u - re1) ^ 0x80808080u;
            o.a[a] = v8i{(int)re0, (int)re1, (int)im0, (int)im1, (int)n0, (int)n1, 0, 0};
        }
#pragma unroll
        for (int b = 0; b < Layout<NW>::BW; ++b) {
            const uint32_t x0 = (uint32_t)r.b[b].x, x1 = (uint32_t)r.b[b].y;
            const uint32_t h0 = (x0 >> 1) & 0x78787878u, h1 = (x1 >> 1) & 0x78787878u;   // 8 x high nibble
            const uint32_t l0 = (x0 << 3) & 0x78787878u, l1 = (x1 << 3) & 0x78787878u;   // 8 x low nibble
            o.b[b] = RE_LOW ? v4i{(int)l0, (int)l1, (int)h0, (int)h1} : v4i{(int)h0, (int)h1, (int)l0, (int)l1};
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const uint32_t x0 = (uint32_t)r.a[a].x, x1 = (uint32_t)r.a[a].y;
        const uint32_t s0 = x0 << 4, s1 = x1 << 4;
        const uint32_t h0 = (x0 ^ 0x88888888u) & 0xF0F0F0F0u, h1 = (x1 ^ 0x88888888u) & 0xF0F0F0F0u;
        const uint32_t l0 = (s0 ^ 0x80808080u) & 0xF0F0F0F0u, l1 = (s1 ^ 0x80808080u) & 0xF0F0F0F0u;
        if (RE_LOW) {
            const uint32_t n0 = (s0 ^ 0x70707070u) & 0xF0F0F0F0u, n1 = (s1 ^ 0x70707070u) & 0xF0F0F0F0u;
            o.a[a] = v8i{(int)l0, (int)l1, (int)h0, (int)h1, (int)n0, (int)n1, 0, 0};
        } else {
            const uint32_t n0 = (x0 ^ 0x77777777u) & 0xF0F0F0F0u, n1 = (x1 ^ 0x77777777u) & 0xF0F0F0F0u;
            o.a[a] = v8i{(int)h0, (int)h1, (int)l0, (int)l1, (int)n0, (int)n1, 0, 0};
        }
    }
#pragma unroll
    for (int b = 0; b < Layout<NW>::BW; ++b) {
        const uint32_t x0 = (uint32_t)r.b[b].x, x1 = (uint32_t)r.b[b].y;
        const uint32_t h0 = (x0 ^ 0x88888888u) & 0xF0F0F0F0u, h1 = (x1 ^ 0x88888888u) & 0xF0F0F0F0u;
        const uint32_t l0 = ((x0 << 4) ^ 0x80808080u) & 0xF0F0F0F0u;
        const uint32_t l1 = ((x1 << 4) ^ 0x80808080u) & 0xF0F0F0F0u;
        o.b[b] = RE_LOW ? v4i{(int)l0, (int)l1, (int)h0, (int)h1} : v4i{(int)h0, (int)h1, (int)l0, (int)l1};
    }
}

// Pre-sums of the unsigned form from the operands a wave multiplies: per A
// block, this lane's row (lane % 32) over the k-step's samples it holds,
// real nibbles (words 0, 1) and imaginary ones (words 2, 3), each a byte
// sum by v_dot4_u32_u8 against ones.
struct PreSum {
    uint32_t r[2], i[2];
};
template <int NW> __device__ __forceinline__ void presum_k(PreSum &ps, const Ops<NW> &o)
{
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        ps.r[a] = __builtin_amdgcn_udot4((uint32_t)o.a[a][0], 0x01010101u, ps.r[a], false);
        ps.r[a] = __builtin_amdgcn_udot4((uint32_t)o.a[a][1], 0x01010101u, ps.r[a], false);
        ps.i[a] = __builtin_amdgcn_udot4((uint32_t)o.a[a][2], 0x01010101u, ps.i[a], false);
        ps.i[a] = __builtin_amdgcn_udot4((uint32_t)o.a[a][3], 0x01010101u, ps.i[a], false);
    }
}

// DIAG: the wave's 2 x 2 blocks sit on the diagonal (eight waves, rows
// 64 wa.. against columns 64 wa.. of a diagonal tile); block (1, 0) lies
// strictly below it and is skipped.
template <int NW, bool DIAG> __device__ __forceinline__ constexpr bool skip_block(int a, int b)
{
    return DIAG && a == 1 && b == 0;
}

// The real products of a k-step first, then the imaginary ones: measured a
// little faster than alternating them (the chip runs at its power limit, and
// this order drew less).
//
// FP8 form: the products of two k-steps at once on
// v_mfma_f32_32x32x64_f8f6f4 (E4M3 on both sides, no block scale), whose
// 32-byte operands are the two k-steps' unpacked words side by side: real
// [R | I | R' | I'] . [R | I | R' | I'], imaginary [I | -R | I' | -R'] .
// [R | I | R' | I'].  All real products of the pair first, then the
// imaginary ones, so that no product waits for the one before it.
template <int NW, bool DIAG>
__device__ __forceinline__ void mfma_pair(Acc<NW, true> &acc, const Ops<NW> &o0, const Ops<NW> &o1)
{
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int b = 0; b < Layout<NW>::BW; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (skip_block<NW, DIAG>(a, b)) continue;
                const int w = 2 * p;   // real: words 0..3, imaginary: words 2..5
                const v8i av = {o0.a[a][w], o0.a[a][w + 1], o0.a[a][w + 2], o0.a[a][w + 3],
                                o1.a[a][w], o1.a[a][w + 1], o1.a[a][w + 2], o1.a[a][w + 3]};
                const v8i bv = {o0.b[b][0], o0.b[b][1], o0.b[b][2], o0.b[b][3],
                                o1.b[b][0], o1.b[b][1], o1.b[b][2], o1.b[b][3]};
                v16f &c = p == 0 ? acc.re[a][b] : acc.im[a][b];
                c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 0, 0, 0);
            }
}

template <int NW, bool DIAG>
__device__ __forceinline__ void mfma_k(Acc<NW, false> &acc, const Ops<NW> &o)
{
#pragma unroll
    for (int b = 0; b < Layout<NW>::BW; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (skip_block<NW, DIAG>(a, b)) continue;
            const v4i re_a = __builtin_shufflevector(o.a[a], o.a[a], 0, 1, 2, 3);
            acc.re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a, o.b[b], acc.re[a][b], 0, 0, 0);
        }
#pragma unroll
    for (int b = 0; b < Layout<NW>::BW; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (skip_block<NW, DIAG>(a, b)) continue;
            const v4i im_a = __builtin_shufflevector(o.a[a], o.a[a], 2, 3, 4, 5);
            acc.im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a, o.b[b], acc.im[a][b], 0, 0, 0);
        }
}

// Instruction order of a k-step: the MFMAs, each followed by a share of the
// unpack of the next k-step (which the matrix core's 32-cycle MFMAs hide)
// and, after the first few, one of the LDS reads of a later k-step -- spread
// out rather than issued as a burst that would stall the wave at issue.
template <int NW, bool DIAG>
__device__ __forceinline__ void kstep_schedule()
{
    using L = Layout<NW>;
    constexpr int MFMAS = L::MFMA_PER_K - (DIAG ? 2 : 0);
    constexpr int VALU = DIAG ? (L::VALU_PER_MFMA * L::MFMA_PER_K + MFMAS - 1) / MFMAS : L::VALU_PER_MFMA;
#pragma unroll
    for (int m = 0; m < MFMAS; ++m) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        if (m < L::READS_PER_K) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
        __builtin_amdgcn_sched_group_barrier(0x002, VALU, 0);   // VALU
    }
}

template <int NW>
__device__ __forceinline__ void wait_stage_and_sync()
{
    // this wave's loads of the next stage have landed (AHEAD - 1 newer
    // stages in flight) and its LDS reads are done; the barrier extends both
    // to the workgroup
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT((AHEAD - 1) * Layout<NW>::DMA_PER_WAVE));
    __builtin_amdgcn_s_waitcnt(XENG_LGKMCNT0);
    __syncthreads();
}

// One piece, software-pipelined over its stages.  Entering iteration s, the
// unpacked operands of (s, k-step 0) and the raw data of (s, 1) are in
// registers; the iteration reads (s, 2), (s, 3), (s+1, 0), (s+1, 1) and
// unpacks one k-step ahead of its MFMAs.  The DMA of stage s + AHEAD goes
// into the slot stage s - 1 used, which every wave finished reading before
// the barrier of iteration s - 1; that barrier sits before the first read of
// stage s.  The last iteration's reads of "stage ns" touch a slot whose
// contents are never used.
//
// In the unsigned form the waves on the diagonal (DIAG) also add up the
// nibbles of their A rows into `ps`, at the k-steps they multiply (the
// reads of "stage ns" never count).
template <int NW, bool RE_LOW, bool DIAG, bool U, bool F>
__device__ __forceinline__ void run_piece(Acc<NW, F> &acc, PreSum &ps, uint32_t ring, const Tile &tl, int wave,
                                          int lane, uint32_t a_lane, uint32_t b_lane)
{
    constexpr bool SUMS = U && DIAG;
    const int ns = (tl.t1 - tl.t0 + STAGE - 1) / STAGE;
    DmaLane<NW> dl;
    dma_lane_setup<NW>(dl, tl, wave, lane);
    // nothing else in flight: the ring's vmcnt waits then count DMA only
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) issue_stage<NW>(ring + d * SLOT, tl, dl, d, wave, lane);
    wait_stage_and_sync<NW>();

    Raw<NW> r0, r1;
    Ops<NW> u0, u1;
    if constexpr (F) {
        // FP8: a k-step pair at a time.  Entering each half stage, the raw
        // data of its two k-steps is in r0, r1; both are unpacked, the next
        // pair's reads are issued, then the pair's products.
        {
            const lds_u8 *pa = (const lds_u8 *)(uintptr_t)(ring + a_lane);
            const lds_u8 *pb = (const lds_u8 *)(uintptr_t)(ring + b_lane);
            read_k<NW>(r0, pa, pb, 0);
            read_k<NW>(r1, pa, pb, 1);
        }
        int cur = 0;
        for (int s = 0; s < ns; ++s) {
            const int nxt = cur == NSLOT - 1 ? 0 : cur + 1;
            const int iss = cur == 0 ? NSLOT - 1 : cur - 1;
            issue_stage<NW>(ring + iss * SLOT, tl, dl, s + AHEAD, wave, lane);
            const lds_u8 *pa = (const lds_u8 *)(uintptr_t)(ring + cur * SLOT + a_lane);
            const lds_u8 *pb = (const lds_u8 *)(uintptr_t)(ring + cur * SLOT + b_lane);
            const lds_u8 *qa = (const lds_u8 *)(uintptr_t)(ring + nxt * SLOT + a_lane);
            const lds_u8 *qb = (const lds_u8 *)(uintptr_t)(ring + nxt * SLOT + b_lane);
            __builtin_amdgcn_sched_barrier(0);
            // k-steps 0, 1
            unpack_k<NW, RE_LOW, U, F>(u0, r0);
            unpack_k<NW, RE_LOW, U, F>(u1, r1);
            read_k<NW>(r0, pa, pb, 2);
            read_k<NW>(r1, pa, pb, 3);
            mfma_pair<NW, DIAG>(acc, u0, u1);
            if constexpr (SUMS) {
                presum_k<NW>(ps, u0);
                presum_k<NW>(ps, u1);
            }
            __builtin_amdgcn_sched_barrier(0);
            // k-steps 2, 3; stage s + 1 must be in LDS before its first read
            unpack_k<NW, RE_LOW, U, F>(u0, r0);
            unpack_k<NW, RE_LOW, U, F>(u1, r1);
            wait_stage_and_sync<NW>();
            read_k<NW>(r0, qa, qb, 0);
            read_k<NW>(r1, qa, qb, 1);
            mfma_pair<NW, DIAG>(acc, u0, u1);
            if constexpr (SUMS) {
                presum_k<NW>(ps, u0);
                presum_k<NW>(ps, u1);
            }
            __builtin_amdgcn_sched_barrier(0);
            cur = nxt;
        }
        __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
        __syncthreads();       // the next piece's DMA reuses the slots
    } else {
        {
            const lds_u8 *pa = (const lds_u8 *)(uintptr_t)(ring + a_lane);
            const lds_u8 *pb = (const lds_u8 *)(uintptr_t)(ring + b_lane);
            read_k<NW>(r0, pa, pb, 0);
            read_k<NW>(r1, pa, pb, 1);
            unpack_k<NW, RE_LOW, U, F>(u0, r0);
        }
        int cur = 0;    // slot of stage s
        for (int s = 0; s < ns; ++s) {
            const int nxt = cur == NSLOT - 1 ? 0 : cur + 1;
            const int iss = cur == 0 ? NSLOT - 1 : cur - 1;   // slot of stage s - 1 = s + AHEAD
            issue_stage<NW>(ring + iss * SLOT, tl, dl, s + AHEAD, wave, lane);
            const lds_u8 *pa = (const lds_u8 *)(uintptr_t)(ring + cur * SLOT + a_lane);
            const lds_u8 *pb = (const lds_u8 *)(uintptr_t)(ring + cur * SLOT + b_lane);
            const lds_u8 *qa = (const lds_u8 *)(uintptr_t)(ring + nxt * SLOT + a_lane);
            const lds_u8 *qb = (const lds_u8 *)(uintptr_t)(ring + nxt * SLOT + b_lane);
            __builtin_amdgcn_sched_barrier(0);
            // k-step 0
            read_k<NW>(r0, pa, pb, 2);
            unpack_k<NW, RE_LOW, U, F>(u1, r1);
            mfma_k<NW, DIAG>(acc, u0);
            if constexpr (SUMS) presum_k<NW>(ps, u0);
            kstep_schedule<NW, DIAG>();
            __builtin_amdgcn_sched_barrier(0);
            // k-step 1
            read_k<NW>(r1, pa, pb, 3);
            unpack_k<NW, RE_LOW, U, F>(u0, r0);
            mfma_k<NW, DIAG>(acc, u1);
            if constexpr (SUMS) presum_k<NW>(ps, u1);
            kstep_schedule<NW, DIAG>();
            __builtin_amdgcn_sched_barrier(0);
            // k-step 2: stage s + 1 must be in LDS before its first read
            wait_stage_and_sync<NW>();
            read_k<NW>(r0, qa, qb, 0);
            unpack_k<NW, RE_LOW, U, F>(u1, r1);
            mfma_k<NW, DIAG>(acc, u0);
            if constexpr (SUMS) presum_k<NW>(ps, u0);
            kstep_schedule<NW, DIAG>();
            __builtin_amdgcn_sched_barrier(0);
            // k-step 3
            read_k<NW>(r1, qa, qb, 1);
            unpack_k<NW, RE_LOW, U, F>(u0, r0);
            mfma_k<NW, DIAG>(acc, u1);
            if constexpr (SUMS) presum_k<NW>(ps, u1);
            kstep_schedule<NW, DIAG>();
            __builtin_amdgcn_sched_barrier(0);
            cur = nxt;
        }
        __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
        __syncthreads();       // the next piece's DMA reuses the slots
    }
}

// A wave whose accumulator region lies wholly below the diagonal: its
// products would never be stored, so it computes nothing (which also spares
// the power that work would draw), but it keeps its share of the
// workgroup's DMA and passes the same barriers as run_piece.
template <int NW>
__device__ __forceinline__ void idle_piece(uint32_t ring, const Tile &tl, int wave, int lane)
{
    const int ns = (tl.t1 - tl.t0 + STAGE - 1) / STAGE;
    DmaLane<NW> dl;
    dma_lane_setup<NW>(dl, tl, wave, lane);
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) issue_stage<NW>(ring + d * SLOT, tl, dl, d, wave, lane);
    wait_stage_and_sync<NW>();
    int cur = 0;
    for (int s = 0; s < ns; ++s) {
        const int iss = cur == 0 ? NSLOT - 1 : cur - 1;
        issue_stage<NW>(ring + iss * SLOT, tl, dl, s + AHEAD, wave, lane);
        wait_stage_and_sync<NW>();
        cur = cur == NSLOT - 1 ? 0 : cur + 1;
    }
    __builtin_amdgcn_s_waitcnt(XENG_VMCNT(0));
    __syncthreads();
}

// Accumulators hold 256x the stored values (both operands carry 16x the
// sample parts), so a flush adds acc >> 8; every value is a multiple of
// 256, so this is exact.  Pairs go to the slot as packed 64-bit words (see
// the layout note): a tile shared with other pieces takes one 64-bit atomic
// add per pair.
//
// FP8 accumulators hold the integer sums x 2^-18 (each operand carries
// 2^-9), below 2^24 in magnitude: scaling by 2^18 recovers them exactly.
template <int SHIFT> __device__ __forceinline__ int32_t acc_val(int32_t v) { return v >> SHIFT; }
template <int SHIFT> __device__ __forceinline__ int32_t acc_val(float v) { return (int32_t)(v * 262144.0f); }

template <int SHIFT, typename V>
__device__ __forceinline__ void flush_atomic(gw64 *blk, const V &re, const V &im)
{
#pragma unroll
    for (int r = 0; r < 16; ++r)
        __hip_atomic_fetch_add(blk + r * 64, pack_pair(acc_val<SHIFT>(re[r]), acc_val<SHIFT>(im[r])),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole-tile flush of one wave's 2 x BW blocks (column blocks cb0..): stores
// if the slot holds zeros, else read-modify-write with the loads of a row of
// blocks issued together (one memory latency per row, not one per value).
template <int NW, int SHIFT, bool F>
__device__ __forceinline__ void flush_owned(gw64 *tb, const Acc<NW, F> &acc, int wa, int cb0, bool fresh)
{
    constexpr int BW = Layout<NW>::BW;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        gw64 *blk[BW];
#pragma unroll
        for (int b = 0; b < BW; ++b) blk[b] = tb + ((2 * wa + a) * BLKS + cb0 + b) * BLOCK_W;
        uint64_t old[BW][16];
#pragma unroll
        for (int b = 0; b < BW; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) old[b][r] = fresh ? 0 : blk[b][r * 64];
#pragma unroll
        for (int b = 0; b < BW; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                blk[b][r * 64] =
                    old[b][r] + pack_pair(acc_val<SHIFT>(acc.re[a][b][r]), acc_val<SHIFT>(acc.im[a][b][r]));
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Persistent kernel: workgroup w runs pieces [wg_off[w], wg_off[w+1]).  A
// piece's tile field holds (I, J2): A rows 128 I.., B columns 256 J2.., i.e.
// accumulator tiles (I, 2 J2) and (I, 2 J2 + 1) where they are in the upper
// triangle.  U: the unsigned form; F (with U): its FP8 products.
template <int NW, bool U = false, bool F = false>
__global__ __launch_bounds__(64 * NW, 1) void xcorr_dma(KernelArgs args)
{
    static_assert(U || !F, "the FP8 form multiplies the unsigned nibbles");
    using L = Layout<NW>;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    // a prepared batch's device guard refused this launch
    if (args.skip != nullptr && *args.skip != 0) return;
    // LDS byte address of the ring, wave-uniform (scalar register)
    const uint32_t ring = (uint32_t)__builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wave-uniform, so that everything derived from it stays scalar
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // per-lane parts of the transposed-read addresses (see read_k); the
    // wave's region adds to them per piece
    const int grp = lane >> 4, jl = lane & 15;
    const uint32_t a_lane0 = GRP_A * (grp >> 1) + 128 * (grp & 1) + 8 * jl;
    const uint32_t b_lane0 = A_STAGE + GRP_B * (grp >> 1) + 128 * (grp & 1) + 8 * jl;

    // clock probe (measurement only): workgroup 0's start and end
    const bool stamp = args.clock != nullptr && blockIdx.x == 0 && tid == 0;
    if (stamp) {
        args.clock[0] = (int64_t)__builtin_amdgcn_s_memtime();
        args.clock[1] = (int64_t)__builtin_amdgcn_s_memrealtime();
    }
    const int p_begin = args.wg_off[blockIdx.x], p_end = args.wg_off[blockIdx.x + 1];
    for (int pi = p_begin; pi < p_end; ++pi) {
        const Piece pce = args.pieces[pi];
        const JobDesc jd = args.jobs ? args.jobs[pce.job] : args.job0;
        const int ti = pce.tile & 0xFFFF, tj2 = (pce.tile >> 16) & 0xFFFF;
        const bool atomic = pce.t1_atomic < 0;
        // every field is wave-uniform: keep them in scalar registers
        Tile tl;
        tl.samples = uniform(jd.samples);
        tl.zeros = uniform(args.zeros);
        tl.stride = uniform(jd.stride);
        tl.n = __builtin_amdgcn_readfirstlane(jd.n);
        tl.row0 = __builtin_amdgcn_readfirstlane(ti * WA_ROWS);
        tl.col0 = __builtin_amdgcn_readfirstlane(tj2 * WB_COLS);
        tl.t0 = __builtin_amdgcn_readfirstlane(pce.t0);
        tl.t1 = __builtin_amdgcn_readfirstlane(pce.t1_atomic & 0x7FFFFFFF);
        // this wave's region: rows 64 wa.. of the A block against column
        // blocks of the B block.  The waves of a workgroup run on SIMD
        // wave % 4.  Where one tile of the window is not in the triangle
        // (below the diagonal: the window of an odd tile row that starts one
        // tile left of it; or past the last tile column), four of the eight
        // regions have no work; the region map then puts the other four on
        // four different SIMDs instead of two waves each on two of them,
        // halving the matrix time of such a window's stages.
        int wa = wave / L::WB_WAVES, wb = wave % L::WB_WAVES;
        if constexpr (NW == 8) {
            const int tjl = 2 * tj2, tjr = tjl + 1;
            const bool vl = tjl >= ti && tjl < jd.nt, vr = tjr >= ti && tjr < jd.nt;
            if (vr && !vl && wa == 0) wb ^= 2;
            if (vl && !vr && wa == 1) wb ^= 2;
        }
        const uint32_t a_lane = a_lane0 + 512 * wa, b_lane = b_lane0 + 256 * L::BW * wb;
        // this wave's accumulator tile; a region wholly below the diagonal
        // is neither computed nor stored (the wave stays in step for the
        // workgroup's DMA and barriers)
        const int tj = 2 * tj2 + wb / (L::WB_WAVES / 2);
        const int cb0 = (wb % (L::WB_WAVES / 2)) * L::BW;   // first column block in the tile
        const bool valid = tj >= ti && tj < jd.nt;
        // rows 64 wa.. of tile ti against columns 32 cb0 .. 32 (cb0 + BW) - 1
        // of tile tj: wholly below the diagonal?
        const bool below = WA_ROWS * (tj - ti) + BLK * (cb0 + L::BW) <= 64 * wa;
        // or wholly past the last input (rows or columns >= N: never
        // exported; small N and the edge tiles of N not a multiple of 256)
        const bool outside = WA_ROWS * ti + 64 * wa >= jd.n || WA_ROWS * tj + BLK * cb0 >= jd.n;

        Acc<NW, F> acc;
        PreSum ps = {{0u, 0u}, {0u, 0u}};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < L::BW; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc.re[a][b][r] = 0;
                    acc.im[a][b][r] = 0;
                }
        // eight waves: a 64 x 64 region on the diagonal skips its block below it
        const bool diag = NW == 8 && tj == ti && cb0 == 2 * wa;
        // a wave whose tile lies past the last tile column (odd tile count)
        // has nothing to compute either
        if (below || outside || tj >= jd.nt)
            idle_piece<NW>(ring, tl, wave, lane);
        else if (jd.flags & JOB_RE_LOW) {
            if (diag)
                run_piece<NW, true, true, U, F>(acc, ps, ring, tl, wave, lane, a_lane, b_lane);
            else
                run_piece<NW, true, false, U, F>(acc, ps, ring, tl, wave, lane, a_lane, b_lane);
        } else {
            if (diag)
                run_piece<NW, false, true, U, F>(acc, ps, ring, tl, wave, lane, a_lane, b_lane);
            else
                run_piece<NW, false, false, U, F>(acc, ps, ring, tl, wave, lane, a_lane, b_lane);
        }

        // unsigned form: the diagonal waves of a job's tiles see every A
        // row of the job over every sample exactly once (each window's
        // pieces split its samples; a diagonal wave is never idle while its
        // rows hold inputs), so their nibble sums are the job's pre-sums;
        // lanes l and l + 32 hold the same row
        if constexpr (U) {
            int32_t *const presum = args.presum != nullptr ? args.presum : jd.presum;
            if (diag && presum != nullptr && !outside) {
                const int n4 = (jd.n + 3) & ~3;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const uint32_t r = ps.r[a] + (uint32_t)__shfl_xor((int)ps.r[a], 32);
                    const uint32_t i = ps.i[a] + (uint32_t)__shfl_xor((int)ps.i[a], 32);
                    const int row = WA_ROWS * ti + 64 * wa + 32 * a + lane;
                    if (lane < 32 && row < jd.n) {
                        __hip_atomic_fetch_add(presum + row, (int32_t)r, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_add(presum + n4 + row, (int32_t)i, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }

        if (valid && !below && !outside) {
            // the sums carry 256x the values (both operands 16x), or 8x in
            // the unsigned form (the FP8 form's scale is undone in acc_val)
            constexpr int SHIFT = U ? 3 : 8;
            const int64_t tile_idx = (int64_t)ti * jd.nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
            gw64 *tb = (gw64 *)(jd.acc + tile_idx * TILE_I32) + lane;
            if (atomic) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < L::BW; ++b) {
                        if (diag && a == 1 && b == 0) continue;   // below the diagonal, never computed
                        flush_atomic<SHIFT>(tb + ((2 * wa + a) * BLKS + cb0 + b) * BLOCK_W, acc.re[a][b],
                                            acc.im[a][b]);
                        // one block at a time: keeps the register file for the main loop
                        __builtin_amdgcn_sched_barrier(0);
                    }
            } else if (jd.flags & JOB_FRESH) {
                flush_owned<NW, SHIFT, F>(tb, acc, wa, cb0, true);
            } else {
                flush_owned<NW, SHIFT, F>(tb, acc, wa, cb0, false);
            }
        }
    }
    if (stamp) {
        args.clock[2] = (int64_t)__builtin_amdgcn_s_memtime();
        args.clock[3] = (int64_t)__builtin_amdgcn_s_memrealtime();
    }
}

}  // namespace dma

constexpr int DMA_LDS_BYTES = dma::NSLOT * dma::SLOT;

// Both instances are built: eight waves (two per SIMD, so one wave's
// unpack overlaps the other's matrix work) and four (one per SIMD, four
// column blocks each, fewer transposed reads per multiply).  The launch
// configuration picks one per call.
//
// Once per device, before any launch (and outside any stream capture): the
// kernel's LDS ring exceeds the default dynamic-LDS limit.
hipError_t init_dma_kernel()
{
    hipError_t e = hipFuncSetAttribute((const void *)dma::xcorr_dma<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       DMA_LDS_BYTES);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)dma::xcorr_dma<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                DMA_LDS_BYTES);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)dma::xcorr_dma<8, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                DMA_LDS_BYTES);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)dma::xcorr_dma<8, true, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, DMA_LDS_BYTES);
    return e;
}

// The unsigned form (pre-sum path): eight waves, int8 or (fp8) FP8
// products; `a.zeros` must then point at zero bytes (nibbles u = 0), the
// zero sample of that form.  FP8 pieces must stay within
// MAX_PIECE_STAGES_FP8_UNSIGNED stages.
hipError_t launch_correlate_dma_unsigned(const KernelArgs &a, int grid, bool fp8, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (fp8)
        hipLaunchKernelGGL((dma::xcorr_dma<8, true, true>), dim3(grid), dim3(64 * 8), DMA_LDS_BYTES, stream, a);
    else
        hipLaunchKernelGGL((dma::xcorr_dma<8, true>), dim3(grid), dim3(64 * 8), DMA_LDS_BYTES, stream, a);
    return hipGetLastError();
}

hipError_t launch_correlate_dma(const KernelArgs &a, int grid, int waves, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (waves == 4)
        hipLaunchKernelGGL(dma::xcorr_dma<4>, dim3(grid), dim3(64 * 4), DMA_LDS_BYTES, stream, a);
    else
        hipLaunchKernelGGL(dma::xcorr_dma<8>, dim3(grid), dim3(64 * 8), DMA_LDS_BYTES, stream, a);
    return hipGetLastError();
}

}  // namespace xeng
