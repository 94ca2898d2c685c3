// gfx950 kernels of the X-engine correlator.
//
// The hot kernel (xcorr_mfma) computes, for one 128 x 128 tile (ti, tj) of
// the upper triangle and one range of time samples, the visibilities
//   V_ij = sum_t x_i(t) conj(x_j(t))                      (Sec. 2.2, eta)
// of 4+4-bit offset-encoded samples and adds them into int32 accumulators.
//
// The complex product is split into two real int8 contractions over a
// K axis that carries the real parts of a k-step's 16 samples on MFMA lanes
// 0-31 and the imaginary parts on lanes 32-63:
//   Re V = [Re x_i | Im x_i] . [Re x_j | Im x_j]    = Re_i Re_j + Im_i Im_j
//   Im'  = [Im x_i | ~Re x_i] . [Re x_j | Im x_j]   = Im_i Re_j - Re_i Im_j - Im_j
// with ~Re = -Re - 1 (the bitwise complement of the 4-bit value, which,
// unlike -Re, never leaves [-8, 7]).  So the row (A) side keeps three int8
// vectors per sample group (Re, Im, ~Re) and the column (B) side two (Re,
// Im); one B operand feeds both products.  The stored imaginary part is
// Im V_ij - S_j with S_j = sum_t Im x_j(t); as Im V_jj = 0, the diagonal
// holds -S_j and the dump adds it back.  Every partial sum is an exact
// int32.  The DMA kernel stores the same form.
//
// Data path per 32-sample stage (double-buffered in LDS):
//   global (time-major bytes) -> dword loads, 4 inputs x 8 samples per lane
//   -> 4x4 byte transposes (v_perm) -> nibble unpack to int8 -> LDS
//   -> ds_read_b128 operands -> v_mfma_i32_32x32x32_i8.
// The paper's own design packed several low-bit products into 24-bit
// multiply-adds on GCN3 (Sec. 2.3, "GPUs"); on CDNA4 the int8 matrix cores
// do this work instead (Sec. 4.1 anticipates low-bit matrix units).
//
// FP8 instances (an exact matrix-core path on 8-bit floats, Sec. 4.1's
// low-bit matrix units) stage every 4-bit value v in [-8, 7] as its OCP
// E4M3 code (1 sign, 4 exponent bits with bias 7, 3 mantissa bits: every
// integer of magnitude <= 16 is exact, -v included, so the imaginary
// operand is [Im | -Re] and carries no bias) and multiply on
// v_mfma_f32_32x32x16_fp8_fp8 into fp32 accumulators.  Products are
// exact, and fp32 sums of integers are exact while below 2^24: with at most
// 128 per sample, pieces below 2^17 samples flush exact integers, converted
// to int32.
//
// UNSIGNED instances multiply the stored nibbles u = x + 8 themselves (the
// paper's unsigned form, whose O(N) bookkeeping is the pre-sum correction
// of xeng_presum.hip): A = [uR | uI] and [uI | -uR], B = [8 uR | 8 uI], so
// the sums are 8 x sum (uR_i uR_j + uI_i uI_j) and 8 x sum (uI_i uR_j -
// uR_i uI_j), flushed with a shift of 3.  At most 3600 per sample, so such
// pieces stay below 2^19 samples (int32 register sums).
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// LDS stage layout.  A stage is 64 samples = 4 MFMA k-steps.  For each
// k-step q a component region holds 128 tile rows x 16 bytes (the 16
// samples of one input, in time order).  A rows keep Re, Im, ~Re as int8;
// B rows keep 16*Re, 16*Im as int8 (the scale makes their unpack three bit
// operations per four samples; every product is then 16x the true one and
// the flush divides it out exactly).  This is the general kernel, for any
// alignment and N; 16-byte-aligned arrays take the DMA kernel instead.
constexpr int CH = TILE * 16;       // 2048 bytes
constexpr int QSTEPS = STAGE / KSTEP;   // 4
constexpr int A_Q = 3 * CH;
constexpr int B_Q = 2 * CH;
constexpr int A_BYTES = QSTEPS * A_Q;   // 24 KB
constexpr int B_BYTES = QSTEPS * B_Q;   // 16 KB
constexpr int STAGE_BYTES = A_BYTES + B_BYTES;   // 40 KB
constexpr int NBUF = 2;

__device__ __forceinline__ uint32_t vperm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    return __builtin_amdgcn_perm(s0, s1, sel);
}

// 4 x 4 byte transpose: in[t] holds 4 inputs at time t; out[c] holds input
// c at the 4 times (byte = time).
__device__ __forceinline__ void transpose4(uint32_t i0, uint32_t i1, uint32_t i2, uint32_t i3,
                                           uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3)
{
    const uint32_t ab_lo = vperm(i1, i0, 0x05010400u);   // a0 b0 a1 b1
    const uint32_t ab_hi = vperm(i1, i0, 0x07030602u);   // a2 b2 a3 b3
    const uint32_t cd_lo = vperm(i3, i2, 0x05010400u);
    const uint32_t cd_hi = vperm(i3, i2, 0x07030602u);
    o0 = vperm(cd_lo, ab_lo, 0x05040100u);               // a0 b0 c0 d0
    o1 = vperm(cd_lo, ab_lo, 0x07060302u);               // a1 b1 c1 d1
    o2 = vperm(cd_hi, ab_hi, 0x05040100u);
    o3 = vperm(cd_hi, ab_hi, 0x07060302u);
}

// Offset-binary nibbles (0..15, one per byte) -> signed int8 value v = n - 8
// and its complement ~v = -v - 1 = 7 - n, four at a time, with no carries
// between bytes:
//   n - 8 = (n + 0x78) ^ 0x80,   7 - n = (0x87 - n) ^ 0x80.
__device__ __forceinline__ uint32_t nib_to_i8(uint32_t n) { return (n + 0x78787878u) ^ 0x80808080u; }
__device__ __forceinline__ uint32_t nib_to_not_i8(uint32_t n) { return (0x87878787u - n) ^ 0x80808080u; }

// Offset-binary nibbles (0..15, one per byte) -> the E4M3 codes of v = n - 8,
// four at a time.  For n >= 8 the code of v = n - 8 in 0..7 is
// POS[n - 8]; for n < 8, v = -(8 - n) and the code is 0x80 | NEG[n] with
// NEG[n] the code of 8 - n.  Codes: 1 = 0x38 (2^0), 2 = 0x40, 3 = 0x44
// (1.5 x 2), 4 = 0x48, 5 = 0x4A (1.25 x 4), 6 = 0x4C, 7 = 0x4E, 8 = 0x50.
// Each table is eight bytes, read by a byte permute with selector n & 7;
// bit 3 of n picks the table.
constexpr uint32_t E4M3_POS_LO = 0x44403800u, E4M3_POS_HI = 0x4E4C4A48u;   // v = 0, 1, .. 7
constexpr uint32_t E4M3_NEG_LO = 0x4A4C4E50u, E4M3_NEG_HI = 0x38404448u;   // |v| = 8, 7, .. 1
__device__ __forceinline__ uint32_t nib_to_e4m3(uint32_t n)
{
    const uint32_t sel = n & 0x07070707u;
    const uint32_t pos = vperm(E4M3_POS_HI, E4M3_POS_LO, sel);
    const uint32_t neg = vperm(E4M3_NEG_HI, E4M3_NEG_LO, sel) | 0x80808080u;
    const uint32_t hi = ((n >> 3) & 0x01010101u) * 0xFFu;   // 0xFF in the bytes with n >= 8
    return (pos & hi) | (neg & ~hi);
}

// Global-memory views: loads through these pointers are global (not flat)
// instructions, so they only count against the vector-memory counter and
// stay in flight while the LDS reads and MFMAs of the current stage run.
typedef __attribute__((address_space(1))) const u32x2 gcu64;
typedef __attribute__((address_space(1))) const uint8_t gcu8;
// the same eight bytes at any byte address
typedef u32x2 u32x2_u __attribute__((aligned(1)));
typedef __attribute__((address_space(1))) const u32x2_u gcu64u;
typedef __attribute__((address_space(1))) uint64_t gw64;

// One lane's share of a stage: 8 inputs x 8 consecutive samples of one
// block (d[k] = the 8 inputs at sample k), as loaded, plus a mask of which
// samples are real (bit k) -- the others become the zero sample at unpack.
struct StageRegs {
    u32x2 d[8];
    uint32_t valid;
};
constexpr uint32_t ALL_VALID = 0xFFu;

// Per-piece constants of one lane.
struct PieceCtx {
    const uint8_t *samples;
    int64_t stride;
    int n, t0, t1;
    int i0;               // first of the 8 inputs this lane stages
    uint32_t off;         // lane byte offset from a stage's first time row
    bool full_rows;       // all 128 inputs of this lane's block are < n
    int t_lane;           // first sample of this lane inside a stage
};

// Fast stage: every sample and input in range.  Eight 8-byte loads at a
// uniform row base plus a 32-bit lane offset.
__device__ __forceinline__ void load_fast(StageRegs &r, const uint8_t *row0, int64_t stride,
                                          uint32_t off)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) r.d[k] = *(gcu64 *)(row0 + (int64_t)k * stride + off);
    r.valid = ALL_VALID;
}

// Edge stage: the same eight loads with every address clamped into the
// array.  Nothing loaded is consumed here, so the loads of both paths stay
// in flight and the memory-counter waits stay precise.
__device__ __forceinline__ void load_clamped(StageRegs &r, const PieceCtx &pc, int t_first)
{
    const bool vi = pc.i0 < pc.n;
    uint32_t valid = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int t = t_first + k;
        const bool vt = t < pc.t1;
        const uint8_t *row = pc.samples + (int64_t)(vt ? t : pc.t0) * pc.stride;
        r.d[k] = *(gcu64 *)(row + (vi ? pc.i0 : 0));
        valid |= ((vt && vi) ? 1u : 0u) << k;
    }
    r.valid = valid;
}

// Unaligned rows (a base or stride not a multiple of 8, or N not a multiple
// of 8): one 8-byte load per row at any byte address -- global loads run in
// unaligned-access mode, which the compiler also assumes for align-1 loads.
// A lane whose eight inputs cross input N - 1 reads the eight bytes that end
// there and shifts its own down to the bottom, so no load reaches past the
// row's N bytes; the inputs past N become the zero sample.  For N < 8 the
// one lane with inputs reads them byte by byte.
__device__ __forceinline__ void load_unaligned(StageRegs &r, const PieceCtx &pc, int t_first)
{
    constexpr uint64_t ZERO8 = 0x8888888888888888ull;
    const int nb = pc.n - pc.i0;                                  // this lane's inputs that exist
    const int off = min(pc.i0, pc.n - 8);                         // first byte read (n >= 8)
    const uint32_t sh = 8u * (uint32_t)(pc.i0 - off);             // bits below this lane's first input
    const uint64_t keep = nb >= 8 ? ~0ull : nb > 0 ? (1ull << (8 * nb)) - 1 : 0ull;
    uint32_t valid = 0;
    if (pc.n >= 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int t = t_first + k;
            const bool vt = t < pc.t1;
            const uint8_t *row = pc.samples + (int64_t)(vt ? t : pc.t0) * pc.stride;
            uint64_t v = ZERO8;
            if (nb > 0) {
                const u32x2 w = *(gcu64u *)(row + off);
                v = ((((uint64_t)w.y << 32) | w.x) >> sh & keep) | (ZERO8 & ~keep);
            }
            r.d[k] = u32x2{(uint32_t)v, (uint32_t)(v >> 32)};
            valid |= (vt ? 1u : 0u) << k;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int t = t_first + k;
            const bool vt = t < pc.t1;
            const uint8_t *row = pc.samples + (int64_t)(vt ? t : pc.t0) * pc.stride;
            uint64_t v = ZERO8;
            for (int b = 0; b < nb; ++b)
                v = (v & ~(0xFFull << (8 * b))) | ((uint64_t)((gcu8 *)row)[pc.i0 + b] << (8 * b));
            r.d[k] = u32x2{(uint32_t)v, (uint32_t)(v >> 32)};
            valid |= (vt ? 1u : 0u) << k;
        }
    }
    r.valid = valid;
}

template <bool ALIGNED>
__device__ __forceinline__ void load_stage(StageRegs &r, const PieceCtx &pc, int s)
{
    const int ts = pc.t0 + s * STAGE;
    if (!ALIGNED)
        load_unaligned(r, pc, ts + pc.t_lane);
    else if (pc.full_rows && ts + STAGE <= pc.t1)
        load_fast(r, pc.samples + (int64_t)ts * pc.stride, pc.stride, pc.off);
    else
        load_clamped(r, pc, ts + pc.t_lane);
}

// Unpack one lane's share of a stage into the stage buffer.  `slot` is the
// byte offset of this lane's (first input, half) in a component region;
// input c of the lane sits 16 * c bytes further.
template <bool ROLE_A, bool RE_LOW, bool UNSIGNED, bool FP8>
__device__ __forceinline__ void stage_write(uint8_t *region, const StageRegs &r, int slot)
{
    uint32_t lo[8], hi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        lo[k] = r.d[k].x;
        hi[k] = r.d[k].y;
    }
    if (r.valid != ALL_VALID) {     // uniform in the steady state
        // samples past the piece's end (or past N) become the zero sample;
        // in the unsigned form the zero sample u = 8 would add 64 per
        // product, so there they become u = 0, which adds nothing
        const uint32_t fill = UNSIGNED ? 0u : 0x88888888u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool ok = (r.valid >> k) & 1u;
            lo[k] = ok ? lo[k] : fill;
            hi[k] = ok ? hi[k] : fill;
        }
    }
    // p[c][h]: input c, samples 4h..4h+3
    uint32_t p[8][2];
    transpose4(lo[0], lo[1], lo[2], lo[3], p[0][0], p[1][0], p[2][0], p[3][0]);
    transpose4(lo[4], lo[5], lo[6], lo[7], p[0][1], p[1][1], p[2][1], p[3][1]);
    transpose4(hi[0], hi[1], hi[2], hi[3], p[4][0], p[5][0], p[6][0], p[7][0]);
    transpose4(hi[4], hi[5], hi[6], hi[7], p[4][1], p[5][1], p[6][1], p[7][1]);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint8_t *dst = region + slot + 16 * c;
        if (UNSIGNED) {
            // the stored nibbles u in 0..15, no offset removed: A rows keep
            // uR, uI and -uR (per byte (0x80 - u) ^ 0x80, no borrows); B
            // rows 8 uR, 8 uI (at most 120: int8)
            const uint32_t h0 = (p[c][0] >> 4) & 0x0F0F0F0Fu, l0 = p[c][0] & 0x0F0F0F0Fu;
            const uint32_t h1 = (p[c][1] >> 4) & 0x0F0F0F0Fu, l1 = p[c][1] & 0x0F0F0F0Fu;
            const uint32_t re0 = RE_LOW ? l0 : h0, im0 = RE_LOW ? h0 : l0;
            const uint32_t re1 = RE_LOW ? l1 : h1, im1 = RE_LOW ? h1 : l1;
            if (ROLE_A) {
                *(uint2 *)(dst) = make_uint2(re0, re1);
                *(uint2 *)(dst + CH) = make_uint2(im0, im1);
                *(uint2 *)(dst + 2 * CH) =
                    make_uint2((0x80808080u - re0) ^ 0x80808080u, (0x80808080u - re1) ^ 0x80808080u);
            } else {
                *(uint2 *)(dst) = make_uint2(re0 << 3, re1 << 3);
                *(uint2 *)(dst + CH) = make_uint2(im0 << 3, im1 << 3);
            }
            continue;
        }
        if (FP8) {
            // A rows: Re, Im, -Re; B rows: Re, Im (E4M3 codes; -v flips
            // the sign bit, exactly)
            const uint32_t h0 = (p[c][0] >> 4) & 0x0F0F0F0Fu, l0 = p[c][0] & 0x0F0F0F0Fu;
            const uint32_t h1 = (p[c][1] >> 4) & 0x0F0F0F0Fu, l1 = p[c][1] & 0x0F0F0F0Fu;
            const uint32_t re0 = nib_to_e4m3(RE_LOW ? l0 : h0), im0 = nib_to_e4m3(RE_LOW ? h0 : l0);
            const uint32_t re1 = nib_to_e4m3(RE_LOW ? l1 : h1), im1 = nib_to_e4m3(RE_LOW ? h1 : l1);
            *(uint2 *)(dst) = make_uint2(re0, re1);
            *(uint2 *)(dst + CH) = make_uint2(im0, im1);
            if (ROLE_A) *(uint2 *)(dst + 2 * CH) = make_uint2(re0 ^ 0x80808080u, re1 ^ 0x80808080u);
            continue;
        }
        if (ROLE_A) {
            const uint32_t h0 = (p[c][0] >> 4) & 0x0F0F0F0Fu, l0 = p[c][0] & 0x0F0F0F0Fu;
            const uint32_t h1 = (p[c][1] >> 4) & 0x0F0F0F0Fu, l1 = p[c][1] & 0x0F0F0F0Fu;
            const uint32_t re0 = RE_LOW ? l0 : h0, im0 = RE_LOW ? h0 : l0;
            const uint32_t re1 = RE_LOW ? l1 : h1, im1 = RE_LOW ? h1 : l1;
            *(uint2 *)(dst) = make_uint2(nib_to_i8(re0), nib_to_i8(re1));
            *(uint2 *)(dst + CH) = make_uint2(nib_to_i8(im0), nib_to_i8(im1));
            *(uint2 *)(dst + 2 * CH) = make_uint2(nib_to_not_i8(re0), nib_to_not_i8(re1));
        } else {
            // flipping bit 3 of an offset-binary nibble gives its 4-bit two's
            // complement; in the high half of a byte that is 16x the value
            const uint32_t x0 = p[c][0] ^ 0x88888888u, x1 = p[c][1] ^ 0x88888888u;
            const uint32_t xh0 = x0 & 0xF0F0F0F0u, xl0 = (x0 << 4) & 0xF0F0F0F0u;
            const uint32_t xh1 = x1 & 0xF0F0F0F0u, xl1 = (x1 << 4) & 0xF0F0F0F0u;
            *(uint2 *)(dst) = RE_LOW ? make_uint2(xl0, xl1) : make_uint2(xh0, xh1);
            *(uint2 *)(dst + CH) = RE_LOW ? make_uint2(xh0, xh1) : make_uint2(xl0, xl1);
        }
    }
}

__device__ __forceinline__ v4i lds128(const uint8_t *p) { return *(const v4i *)p; }

// An accumulator register as the integer it holds (fp32 sums of the FP8
// instances are exact integers below 2^24).
__device__ __forceinline__ int32_t acc_int(int32_t v) { return v; }
__device__ __forceinline__ int32_t acc_int(float v) { return (int32_t)v; }

// Accumulators hold 16x the stored values (B operands are scaled by 16), so
// the flush adds acc >> 4; every value is a multiple of 16, so this is
// exact.  Pairs go to the slot as packed 64-bit words (see the layout note):
// a shared tile takes one 64-bit atomic add per pair.
template <int SHIFT, typename V>
__device__ __forceinline__ void flush_block(gw64 *blk, const V &re, const V &im)
{
#pragma unroll
    for (int r = 0; r < 16; ++r)
        __hip_atomic_fetch_add(blk + r * 64, pack_pair(acc_int(re[r]) >> SHIFT, acc_int(im[r]) >> SHIFT),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool FP8> struct AccT {
    v16i re[2][2];
    v16i im[2][2];
};
template <> struct AccT<true> {
    v16f re[2][2];
    v16f im[2][2];
};
typedef AccT<false> Acc;


// Whole-tile flush of one wave's 2 x 2 blocks: stores if the slot holds
// zeros, else read-modify-write with the loads of a row of blocks issued
// before their stores (one memory latency per row, not one per value).
template <int SHIFT, bool FP8>
__device__ __forceinline__ void flush_owned(gw64 *tb, const AccT<FP8> &acc, int wa, int wb, bool fresh)
{
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        gw64 *blk[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) blk[b] = tb + ((2 * wa + a) * BLKS + (2 * wb + b)) * BLOCK_W;
        uint64_t old[2][16];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) old[b][r] = fresh ? 0 : blk[b][r * 64];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                blk[b][r * 64] =
                    old[b][r] + pack_pair(acc_int(acc.re[a][b][r]) >> SHIFT, acc_int(acc.im[a][b][r]) >> SHIFT);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The FP8 form of a k-step's products: each 16-byte operand is two 8-byte
// E4M3 operands of v_mfma_f32_32x32x16_fp8_fp8 (samples 0..7 of the
// k-step's Re and Im halves, then samples 8..15).
__device__ __forceinline__ v16f mfma_fp8(const v4i &a, const v4i &b, v16f c)
{
    const long a0 = (long)(((uint64_t)(uint32_t)a.y << 32) | (uint32_t)a.x);
    const long a1 = (long)(((uint64_t)(uint32_t)a.w << 32) | (uint32_t)a.z);
    const long b0 = (long)(((uint64_t)(uint32_t)b.y << 32) | (uint32_t)b.x);
    const long b1 = (long)(((uint64_t)(uint32_t)b.w << 32) | (uint32_t)b.z);
    c = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a0, b0, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a1, b1, c, 0, 0, 0);
}

__device__ __forceinline__ v16i mfma_k(const v4i &a, const v4i &b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mfma_k(const v4i &a, const v4i &b, v16f c) { return mfma_fp8(a, b, c); }

// The 32 MFMAs of one stage (4 k-steps x 2 x 2 blocks x Re/Im) on `buf`
// (64 for the FP8 instances, two per block and k-step).
template <bool FP8>
__device__ __forceinline__ void stage_mfma(AccT<FP8> &acc, const uint8_t *buf, int lane, int wa, int wb)
{
#pragma unroll
    for (int q = 0; q < QSTEPS; ++q) {
        const uint8_t *aq = buf + q * A_Q + (lane >> 5) * CH + 16 * (lane & 31);
        const v4i re_a0 = lds128(aq + 512 * (2 * wa));
        const v4i re_a1 = lds128(aq + 512 * (2 * wa + 1));
        const v4i im_a0 = lds128(aq + CH + 512 * (2 * wa));
        const v4i im_a1 = lds128(aq + CH + 512 * (2 * wa + 1));
        const uint8_t *bp = buf + A_BYTES + q * B_Q + (lane >> 5) * CH + 16 * (lane & 31);
        const v4i b0 = lds128(bp + 512 * (2 * wb));
        const v4i b1 = lds128(bp + 512 * (2 * wb + 1));
        acc.re[0][0] = mfma_k(re_a0, b0, acc.re[0][0]);
        acc.im[0][0] = mfma_k(im_a0, b0, acc.im[0][0]);
        acc.re[0][1] = mfma_k(re_a0, b1, acc.re[0][1]);
        acc.im[0][1] = mfma_k(im_a0, b1, acc.im[0][1]);
        acc.re[1][0] = mfma_k(re_a1, b0, acc.re[1][0]);
        acc.im[1][0] = mfma_k(im_a1, b0, acc.im[1][0]);
        acc.re[1][1] = mfma_k(re_a1, b1, acc.re[1][1]);
        acc.im[1][1] = mfma_k(im_a1, b1, acc.im[1][1]);
    }
}

// Correlate one piece: tile (ti, tj) over samples [t0, t1).  Stage s is in
// LDS being multiplied while stage s+1 (in registers) is unpacked into the
// other LDS buffer and stage s+2 loads from memory.  Steps run in pairs with
// no early exit: a stage past the end of the piece holds zero samples and
// adds exactly nothing.
template <bool ALIGNED, bool ROLE_A, bool RE_LOW, bool UNSIGNED, bool FP8>
__device__ __forceinline__ void run_piece(AccT<FP8> &acc, uint8_t *smem, const PieceCtx &pc, int lane,
                                          int wa, int wb, int wslot, bool compute)
{
    const int nst = (pc.t1 - pc.t0 + STAGE - 1) / STAGE;
    uint8_t *buf0 = smem, *buf1 = smem + STAGE_BYTES;
    StageRegs r0, r1;

    load_stage<ALIGNED>(r0, pc, 0);
    load_stage<ALIGNED>(r1, pc, 1);
    stage_write<ROLE_A, RE_LOW, UNSIGNED, FP8>(buf0, r0, wslot);
    __syncthreads();

    for (int s = 0; s < nst; s += NBUF) {
        load_stage<ALIGNED>(r0, pc, s + 2);
        if (compute) stage_mfma<FP8>(acc, buf0, lane, wa, wb);
        stage_write<ROLE_A, RE_LOW, UNSIGNED, FP8>(buf1, r1, wslot);
        __syncthreads();
        load_stage<ALIGNED>(r1, pc, s + 3);
        if (compute) stage_mfma<FP8>(acc, buf1, lane, wa, wb);
        stage_write<ROLE_A, RE_LOW, UNSIGNED, FP8>(buf0, r0, wslot);
        __syncthreads();
    }
}

// Persistent correlation kernel: workgroup w runs pieces [wg_off[w], wg_off[w+1]).
// 256 threads = 4 waves; wave (wa, wb) owns MFMA blocks ca in {2wa, 2wa+1},
// cb in {2wb, 2wb+1} of the tile (64 x 64 outputs, Re and Im).  Staging:
// waves 0-1 unpack the A (row) block, waves 2-3 the B (column) block; a lane
// takes 8 inputs x 8 samples (lane bits 0-2 and 4 pick the 8-input group,
// bit 3 the half of a k-step, bit 5 and the wave the k-step).
template <bool ALIGNED, bool UNSIGNED, bool FP8>
__global__ __launch_bounds__(256, 2) void xcorr_mfma(KernelArgs args)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[NBUF * STAGE_BYTES];
    // a prepared batch's device guard refused this launch
    if (args.skip != nullptr && *args.skip != 0) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wb = wave & 1;
    const bool role_a = wave < 2;
    const int g8 = (lane & 7) | (((lane >> 4) & 1) << 3);   // 8-input group 0..15
    const int half = (lane >> 3) & 1;                        // samples 0-7 / 8-15 of a k-step
    const int q = 2 * (wave & 1) + (lane >> 5);              // k-step 0..3
    // LDS byte offset of this lane's (input 8*g8, half, k-step); input c of
    // the lane is 16 * c bytes further
    const int wslot = (role_a ? q * A_Q : A_BYTES + q * B_Q) + 128 * g8 + 8 * half;

    const int p_begin = args.wg_off[blockIdx.x], p_end = args.wg_off[blockIdx.x + 1];
    for (int pi = p_begin; pi < p_end; ++pi) {
        const Piece pce = args.pieces[pi];
        const JobDesc jd = args.jobs ? args.jobs[pce.job] : args.job0;
        const int ti = pce.tile & 0xFFFF, tj = (pce.tile >> 16) & 0xFFFF;
        const bool atomic = pce.t1_atomic < 0;
        const int blk0 = (role_a ? ti : tj) * TILE;

        PieceCtx pc;
        pc.samples = jd.samples;
        pc.stride = jd.stride;
        pc.n = jd.n;
        pc.t0 = pce.t0;
        pc.t1 = pce.t1_atomic & 0x7FFFFFFF;
        pc.i0 = blk0 + 8 * g8;
        pc.t_lane = 16 * q + 8 * half;
        // lane offset from a stage's first row: fits 32 bits (stride <= 2^26)
        pc.off = (uint32_t)(pc.t_lane * jd.stride) + (uint32_t)pc.i0;
        pc.full_rows = blk0 + TILE <= jd.n;

        AccT<FP8> acc;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc.re[a][b][r] = 0;
                    acc.im[a][b][r] = 0;
                }

        const bool re_low = (jd.flags & JOB_RE_LOW) != 0;
        // a wave whose 64 x 64 region lies wholly past the last input (rows
        // or columns >= N, never exported) stages its share but multiplies
        // and flushes nothing
        const bool compute = TILE * ti + 64 * wa < jd.n && TILE * tj + 64 * wb < jd.n;
        if (role_a) {
            if (re_low) run_piece<ALIGNED, true, true, UNSIGNED, FP8>(acc, smem, pc, lane, wa, wb, wslot, compute);
            else run_piece<ALIGNED, true, false, UNSIGNED, FP8>(acc, smem, pc, lane, wa, wb, wslot, compute);
        } else {
            if (re_low) run_piece<ALIGNED, false, true, UNSIGNED, FP8>(acc, smem, pc, lane, wa, wb, wslot, compute);
            else run_piece<ALIGNED, false, false, UNSIGNED, FP8>(acc, smem, pc, lane, wa, wb, wslot, compute);
        }

        // integrate into the slot's accumulators: the signed int8 sums carry
        // 16x the value, the unsigned 8x, the FP8 ones the value itself
        if (!compute) continue;
        constexpr int SHIFT = FP8 ? 0 : UNSIGNED ? 3 : 4;
        const int64_t tile_idx = (int64_t)ti * jd.nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
        gw64 *tb = (gw64 *)(jd.acc + tile_idx * TILE_I32) + lane;
        if (atomic) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    flush_block<SHIFT>(tb + ((2 * wa + a) * BLKS + (2 * wb + b)) * BLOCK_W, acc.re[a][b],
                                acc.im[a][b]);
        } else if (jd.flags & JOB_FRESH) {
            flush_owned<SHIFT, FP8>(tb, acc, wa, wb, true);
        } else {
            flush_owned<SHIFT, FP8>(tb, acc, wa, wb, false);
        }
    }
}

// Word of pair (i <= j) in a slot's tile layout.
__device__ __forceinline__ int64_t acc_word(int i, int j, int nt)
{
    const int ti = i >> 7, tj = j >> 7;
    const int ri = i & 127, rj = j & 127;
    const int ca = ri >> 5, ra = ri & 31, cb = rj >> 5, lb = rj & 31;
    const int reg = 4 * (ra >> 3) + (ra & 3);
    const int ln = lb + 32 * ((ra >> 2) & 1);
    const int64_t tile = (int64_t)ti * nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
    return tile * TILE_W + (ca * BLKS + cb) * BLOCK_W + reg * 64 + ln;
}

// Stored imaginary parts of the diagonal, d[j] = -S_j (see the operand
// note at the top), staged before the tiles are exported and zeroed.
__global__ __launch_bounds__(256) void diag_im(const int32_t *__restrict__ acc, int n, int nt,
                                               int32_t *__restrict__ d)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) d[j] = pair_im(reinterpret_cast<const uint64_t *>(acc)[acc_word(j, j, nt)]);
}

// Accumulators (tile layout) -> packed row-major upper triangle of (Re, Im),
// optionally zeroing the slot in the same pass.  A workgroup takes DUMP_ROWS
// rows of one 32-row block row of tile (ti, tj): blockIdx.y = ti and
// blockIdx.x = (tj - ti) * DUMP_PARTS_PER_TILE + ca * DUMP_PARTS + part.
// Reads: row r of the part is 64 threads, thread c taking the 16 bytes of
// columns 32 (c / 16) + 2 (c % 16) .. + 1 (two consecutive words of one
// accumulator register row, so a row is read as four coalesced 256-byte
// runs), staged in LDS as (Re, Im) pairs.  Writes: consecutive threads take
// consecutive pairs of an output row, 128 pairs (1 KB contiguous) per row.
// Few rows per workgroup keep many small workgroups in flight: the export
// is a single pass over memory, and this form measured twice as fast as
// 32-row workgroups.  The imaginary part of (i, j) is stored as Im V_ij -
// S_j, so d[j] is subtracted (exact in wrapping int32 arithmetic, since
// Im V_ij itself fits).
constexpr int DUMP_PITCH = TILE + 1;   // int2 per staged row (padding spreads banks)
constexpr int DUMP_ROWS = 4;
constexpr int DUMP_PARTS = BLK / DUMP_ROWS;
constexpr int DUMP_PARTS_PER_TILE = 4 * DUMP_PARTS;   // workgroups per tile

// A pending unsigned-form correction (CORR; see presum_correct): per
// input, SR at sums[i] and SI at sums[n4 + i] over the t samples that form
// contributed.  It is added to each staged word in the packed 64-bit form,
// before the word is split into (Re, Im): the uncorrected real part may have
// passed the int32 range, which the split would carry into Im.
struct PendingCorr {
    const int32_t *sums;
    int n4;
    int64_t t;
};
__device__ __forceinline__ uint64_t corr_word(const PendingCorr &pc, int n, int i, int j)
{
    const int64_t ri = i < n ? pc.sums[i] : 0, ii = i < n ? pc.sums[pc.n4 + i] : 0;
    const int64_t rj = j < n ? pc.sums[j] : 0, ij = j < n ? pc.sums[pc.n4 + j] : 0;
    const int64_t d_re = -8 * (ri + ii + rj + ij) + 128 * pc.t;
    const int64_t d_im = 8 * (ri - ii) - 8 * (rj - ij);
    return ((uint64_t)d_im << 32) + (uint64_t)d_re;
}

template <bool CORR = false>
__device__ __forceinline__ void dump_block_row(int32_t *__restrict__ acc, int n, int nt,
                                               const int32_t *__restrict__ d, int32_t *__restrict__ out,
                                               int reset, int bx, int by, int2 *stage,
                                               const PendingCorr &pc = PendingCorr{nullptr, 0, 0})
{
    const int ti = by;
    const int tj = ti + bx / DUMP_PARTS_PER_TILE;
    if (tj >= nt) return;
    const int ca = (bx / DUMP_PARTS) & 3, part = bx % DUMP_PARTS;
    const int t = threadIdx.x;
    const int64_t tile = (int64_t)ti * nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
    {
        const int ri = t >> 6, c = t & 63;
        const int ra = DUMP_ROWS * part + ri;
        const int cb = c >> 4, cj0 = 2 * (c & 15);
        const int reg = 4 * (ra >> 3) + (ra & 3), half = (ra >> 2) & 1;
        uint64_t *base = reinterpret_cast<uint64_t *>(acc) + tile * TILE_W + (ca * BLKS + cb) * BLOCK_W + reg * 64 +
                         32 * half + cj0;
        int4 *pw = reinterpret_cast<int4 *>(base);
        const int4 w = *pw;
        if (reset) *pw = make_int4(0, 0, 0, 0);
        uint64_t w0 = (uint64_t)(uint32_t)w.x | ((uint64_t)(uint32_t)w.y << 32);
        uint64_t w1 = (uint64_t)(uint32_t)w.z | ((uint64_t)(uint32_t)w.w << 32);
        if constexpr (CORR) {
            const int i = TILE * ti + BLK * ca + ra, j0 = TILE * tj + BLK * cb + cj0;
            w0 += corr_word(pc, n, i, j0);
            w1 += corr_word(pc, n, i, j0 + 1);
        }
        int2 *row = stage + ri * DUMP_PITCH + BLK * cb + cj0;
        row[0] = make_int2(pair_re(w0), pair_im(w0));
        row[1] = make_int2(pair_re(w1), pair_im(w1));
    }
    __syncthreads();
    const int col = t & (TILE - 1);
    const int j = TILE * tj + col;
    if (j >= n) return;
    const uint32_t dj = (uint32_t)d[j];
    int2 *o = reinterpret_cast<int2 *>(out);
#pragma unroll
    for (int r = t >> 7; r < DUMP_ROWS; r += 2) {
        const int i = TILE * ti + BLK * ca + DUMP_ROWS * part + r;
        if (i >= n || j < i) continue;
        const int64_t k = (int64_t)i * n - (int64_t)i * (i - 1) / 2 + (j - i);
        const int2 v = stage[r * DUMP_PITCH + col];
        o[k] = make_int2(v.x, (int32_t)((uint32_t)v.y - dj));
    }
}

__global__ __launch_bounds__(256) void vis_dump(int32_t *__restrict__ acc, int n, int nt,
                                                const int32_t *__restrict__ d,
                                                int32_t *__restrict__ out, int reset)
{
    __shared__ int2 stage[DUMP_ROWS * DUMP_PITCH];
    dump_block_row(acc, n, nt, d, out, reset, blockIdx.x, blockIdx.y, stage);
}

// The export of a slot with a pending unsigned-form correction: the
// diagonal words corrected before d[j] is taken (their imaginary part gets
// no correction, their real part may have wrapped), and `other` (the slot's
// second pre-sum buffer, 2 n4 int32, which the next calls of that form will
// use) cleared.  The unsigned form's contributions carry no imaginary bias,
// so d[j] stays that of the signed calls alone.
__global__ __launch_bounds__(256) void diag_im_corr(const int32_t *__restrict__ acc, int n, int nt,
                                                    int32_t *__restrict__ d, PendingCorr pc,
                                                    int32_t *__restrict__ other)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) {
        const uint64_t w = reinterpret_cast<const uint64_t *>(acc)[acc_word(j, j, nt)];
        d[j] = pair_im(w + corr_word(pc, n, j, j));
    }
    if (j < 2 * pc.n4) other[j] = 0;
}

__global__ __launch_bounds__(256) void vis_dump_corr(int32_t *__restrict__ acc, int n, int nt,
                                                     const int32_t *__restrict__ d, int32_t *__restrict__ out,
                                                     int reset, PendingCorr pc)
{
    __shared__ int2 stage[DUMP_ROWS * DUMP_PITCH];
    dump_block_row<true>(acc, n, nt, d, out, reset, blockIdx.x, blockIdx.y, stage, pc);
}

// Batched export: job blockIdx.z of the descriptor table, the grid sized
// for the largest job (workgroups past a smaller job's tiles return).  One
// launch keeps enough block rows in flight to run at memory speed, where one
// export per launch leaves most of the chip waiting on a single wave of
// workgroups.
__global__ __launch_bounds__(256) void diag_im_batch(const DumpDesc *__restrict__ jobs)
{
    const DumpDesc jd = jobs[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < jd.n) jd.diag[j] = pair_im(reinterpret_cast<const uint64_t *>(jd.acc)[acc_word(j, j, jd.nt)]);
}

__global__ __launch_bounds__(256) void vis_dump_batch(const DumpDesc *__restrict__ jobs)
{
    __shared__ int2 stage[DUMP_ROWS * DUMP_PITCH];
    const DumpDesc jd = jobs[blockIdx.z];
    if ((int)blockIdx.y >= jd.nt || (int)blockIdx.x >= DUMP_PARTS_PER_TILE * jd.nt) return;
    dump_block_row(jd.acc, jd.n, jd.nt, jd.diag, jd.out, jd.reset, blockIdx.x, blockIdx.y, stage);
}

// Ingest of host-sourced frames (the streaming server): up to GATHER_MAX
// frames of `words` 16-byte words each, every frame from pinned host memory
// (read over PCIe by the workgroups themselves, no DMA-engine copy) into
// device memory.  Workgroups (x, f) share frame f; each thread keeps eight
// 16-byte loads in flight.
constexpr int GATHER_MAX = 120;
constexpr int GATHER_WGS_PER_FRAME = 4;
typedef unsigned int gv4u __attribute__((ext_vector_type(4)));
struct GatherArgs {
    int32_t n;                       // frames
    int32_t words;                   // 16-byte words per frame
    const gv4u *src[GATHER_MAX];     // device-visible addresses of pinned host frames
    gv4u *dst[GATHER_MAX];
};

__global__ __launch_bounds__(256) void gather_frames(GatherArgs a)
{
    const gv4u *__restrict__ src = a.src[blockIdx.y];
    gv4u *__restrict__ dst = a.dst[blockIdx.y];
    const int step = (int)(blockDim.x * gridDim.x);
    int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    for (; i + 7 * step < a.words; i += 8 * step) {
        gv4u v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = src[i + k * step];
#pragma unroll
        for (int k = 0; k < 8; ++k) dst[i + k * step] = v[k];
    }
    for (; i < a.words; i += step) dst[i] = src[i];
}

// Rows of n samples (any stride and alignment) copied into rows of n16 = n
// rounded up to 16 bytes, padded with zero samples (0x88): a layout the DMA
// kernel reads.  Workgroup t copies row t, one output dword per thread and
// step, consecutive threads on consecutive dwords, so the reads coalesce.
// A dword's four source bytes are read as the one or two aligned dwords that
// hold them (joined by a byte funnel shift); the second is read only when it
// holds a byte of the row, so every load touches an aligned dword with at
// least one byte of the caller's row in it.
__global__ __launch_bounds__(256) void pad_rows(const uint8_t *__restrict__ src, int64_t stride, int n, int n16,
                                                uint8_t *__restrict__ dst)
{
    const int64_t t = blockIdx.x;
    const uint8_t *row = src + t * stride;
    uint32_t *out_row = reinterpret_cast<uint32_t *>(dst + t * n16);
    for (int c0 = 4 * (int)threadIdx.x; c0 < n16; c0 += 4 * 256) {
        uint32_t out = 0x88888888u;
        if (c0 < n) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(row + c0);
            const uint32_t sh = (uint32_t)(a & 3);
            const uint32_t *p = reinterpret_cast<const uint32_t *>(a - sh);
            const int last = min(c0 + 3, n - 1);        // last byte of the row in this dword
            const uint32_t lo = p[0];
            const uint32_t hi = (sh != 0 && c0 + 4 - (int)sh <= last) ? p[1] : 0u;
            uint32_t v = sh ? __builtin_amdgcn_alignbyte(hi, lo, sh) : lo;
            const int valid = last - c0 + 1;
            if (valid < 4) {
                const uint32_t m = 0xFFFFFFFFu >> (8 * (4 - valid));
                v = (v & m) | (0x88888888u & ~m);
            }
            out = v;
        }
        out_row[c0 >> 2] = out;
    }
}

__global__ __launch_bounds__(256) void fill_zero(int4 *__restrict__ p, int64_t n4)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n4;
         k += (int64_t)gridDim.x * 256)
        p[k] = make_int4(0, 0, 0, 0);
}

// Integration guard of a prepared batch, run ahead of its correlation
// launches: if every job's slot can take its samples without passing T_MAX,
// the counters advance and *skip = 0; otherwise nothing changes, *skip = 1
// (the correlation launches then return at once) and *skipped counts the
// refusal.  One workgroup: every thread checks its share of the jobs, the
// verdict is agreed at a barrier before any counter moves, and the jobs'
// counters are distinct (a batch names each slot once), so each thread
// advances its own.
__global__ __launch_bounds__(1024) void batch_guard(const GuardJob *__restrict__ jobs, int n_jobs, int32_t *skip,
                                                    int64_t *skipped)
{
    bool ok = true;
    for (int k = threadIdx.x; k < n_jobs; k += blockDim.x) ok = ok && jobs[k].n <= T_MAX - *jobs[k].count;
    ok = __syncthreads_and(ok ? 1 : 0) != 0;
    if (ok)
        for (int k = threadIdx.x; k < n_jobs; k += blockDim.x) *jobs[k].count += jobs[k].n;
    if (threadIdx.x == 0) {
        if (!ok) *skipped += 1;
        *skip = ok ? 0 : 1;
    }
}

// Stores one value into a device sample counter, in stream order.
__global__ void set_count(int64_t *p, int64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// Scalar reference: one thread per pair (i <= j), int32 sums over t.
__global__ __launch_bounds__(256) void xcorr_scalar(const uint8_t *__restrict__ s, int64_t n_samples,
                                                    int n, int64_t stride, uint32_t re_low,
                                                    int32_t *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t npairs = (int64_t)n * (n + 1) / 2;
    if (k >= npairs) return;
    const double b = 2.0 * n + 1.0;
    int i = (int)floor((b - sqrt(b * b - 8.0 * (double)k)) * 0.5);
    auto row_start = [n](int64_t r) { return r * n - r * (r - 1) / 2; };
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    while (i + 1 < n && row_start(i + 1) <= k) ++i;
    while (i > 0 && row_start(i) > k) --i;
    const int j = i + (int)(k - row_start(i));
    int32_t vr = 0, vi = 0;
    for (int64_t t = 0; t < n_samples; ++t) {
        const uint32_t bi = s[t * stride + i], bj = s[t * stride + j];
        const int hi_i = (int)(bi >> 4) - 8, lo_i = (int)(bi & 15u) - 8;
        const int hi_j = (int)(bj >> 4) - 8, lo_j = (int)(bj & 15u) - 8;
        const int ri = re_low ? lo_i : hi_i, ii = re_low ? hi_i : lo_i;
        const int rj = re_low ? lo_j : hi_j, ij = re_low ? hi_j : lo_j;
        vr += ri * rj + ii * ij;
        vi += ii * rj - ri * ij;
    }
    out[2 * k] = vr;
    out[2 * k + 1] = vi;
}

// ---------------------------------------------------------------------------
// Launchers (host)
// ---------------------------------------------------------------------------
// `aligned`: every job's samples pointer and row stride are multiples of 4
// bytes and its N is a multiple of 4, so whole dwords can be loaded.
hipError_t launch_correlate(const KernelArgs &a, int grid, bool aligned, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (aligned)
        hipLaunchKernelGGL((xcorr_mfma<true, false, false>), dim3(grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((xcorr_mfma<false, false, false>), dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

// The exact FP8 path: the same kernel with E4M3 operands and fp32 sums
// (pieces below 2^17 samples).
hipError_t launch_correlate_fp8(const KernelArgs &a, int grid, bool aligned, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (aligned)
        hipLaunchKernelGGL((xcorr_mfma<true, false, true>), dim3(grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((xcorr_mfma<false, false, true>), dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

// The unsigned-nibble form (xeng_correlate_presum): the same kernel on the
// stored nibbles; its sums need the pre-sum correction below.
hipError_t launch_correlate_unsigned(const KernelArgs &a, int grid, bool aligned, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (aligned)
        hipLaunchKernelGGL((xcorr_mfma<true, true, false>), dim3(grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((xcorr_mfma<false, true, false>), dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_dump(int32_t *acc, int32_t *diag, int n, int nt, int32_t *out, bool reset,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(diag_im, dim3((n + 255) / 256), dim3(256), 0, stream, acc, n, nt, diag);
    hipLaunchKernelGGL(vis_dump, dim3(DUMP_PARTS_PER_TILE * nt, nt), dim3(256), 0, stream, acc, n, nt, diag, out,
                       reset ? 1 : 0);
    return hipGetLastError();
}

// An export that also applies a slot's pending unsigned-form correction
// (`sums`: its SR, SI over `t` samples, n4 apart) and clears `other`.
hipError_t launch_dump_corr(int32_t *acc, int32_t *diag, int n, int nt, int32_t *out, bool reset,
                            const int32_t *sums, int n4, int64_t t, int32_t *other, hipStream_t stream)
{
    const PendingCorr pc{sums, n4, t};
    const int threads = n > 2 * n4 ? n : 2 * n4;
    hipLaunchKernelGGL(diag_im_corr, dim3((threads + 255) / 256), dim3(256), 0, stream, acc, n, nt, diag, pc, other);
    hipLaunchKernelGGL(vis_dump_corr, dim3(DUMP_PARTS_PER_TILE * nt, nt), dim3(256), 0, stream, acc, n, nt, diag,
                       out, reset ? 1 : 0, pc);
    return hipGetLastError();
}

// `d_jobs`: n_jobs descriptors in device memory (n_jobs <= 65535); n_max and
// nt_max: the largest n and nt among them.
hipError_t launch_dump_batch(const DumpDesc *d_jobs, int n_jobs, int n_max, int nt_max, hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(diag_im_batch, dim3((n_max + 255) / 256, n_jobs), dim3(256), 0, stream, d_jobs);
    hipLaunchKernelGGL(vis_dump_batch, dim3(DUMP_PARTS_PER_TILE * nt_max, nt_max, n_jobs), dim3(256), 0, stream,
                       d_jobs);
    return hipGetLastError();
}

// `dst`: rows * n16 bytes, 16-byte aligned; n16 a multiple of 16, >= n.
hipError_t launch_pad_rows(const uint8_t *src, int64_t stride, int n, int64_t rows, int n16, uint8_t *dst,
                           hipStream_t stream)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(pad_rows, dim3((unsigned)rows), dim3(256), 0, stream, src, stride, n, n16, dst);
    return hipGetLastError();
}

// `n` frames of `bytes` each (a multiple of 16, below 2^31), every address
// 16-byte aligned; any number of frames (GATHER_MAX per launch).
hipError_t launch_gather_frames(const uint8_t *const *src, uint8_t *const *dst, int n, int64_t bytes,
                                hipStream_t stream)
{
    for (int f0 = 0; f0 < n; f0 += GATHER_MAX) {
        GatherArgs a;
        a.n = std::min(GATHER_MAX, n - f0);
        a.words = (int32_t)(bytes / 16);
        for (int k = 0; k < a.n; ++k) {
            a.src[k] = reinterpret_cast<const gv4u *>(src[f0 + k]);
            a.dst[k] = reinterpret_cast<gv4u *>(dst[f0 + k]);
        }
        hipLaunchKernelGGL(gather_frames, dim3(GATHER_WGS_PER_FRAME, (unsigned)a.n), dim3(256), 0, stream, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero(int32_t *p, int64_t n_i32, hipStream_t stream)
{
    const int64_t n4 = n_i32 / 4;
    if (n4 <= 0) return hipSuccess;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<int4 *>(p), n4);
    return hipGetLastError();
}

hipError_t launch_batch_guard(const GuardJob *d_jobs, int n_jobs, int32_t *d_skip, int64_t *d_skipped,
                              hipStream_t stream)
{
    const int threads = std::min(1024, std::max(64, (n_jobs + 63) / 64 * 64));
    hipLaunchKernelGGL(batch_guard, dim3(1), dim3(threads), 0, stream, d_jobs, n_jobs, d_skip, d_skipped);
    return hipGetLastError();
}

hipError_t launch_set_count(int64_t *p, int64_t v, hipStream_t stream)
{
    hipLaunchKernelGGL(set_count, dim3(1), dim3(64), 0, stream, p, v);
    return hipGetLastError();
}

hipError_t launch_reference(const uint8_t *s, int64_t n_samples, int n, int64_t stride,
                            uint32_t re_low, int32_t *out, hipStream_t stream)
{
    const int64_t npairs = (int64_t)n * (n + 1) / 2;
    const int64_t blocks = (npairs + 255) / 256;
    hipLaunchKernelGGL(xcorr_scalar, dim3((unsigned)blocks), dim3(256), 0, stream, s, n_samples,
                       n, stride, re_low, out);
    return hipGetLastError();
}

}  // namespace xeng
