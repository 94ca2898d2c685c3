// Flag-aware correlation and its RFI-excision step (the "RFI Excision" task
// of Table tab:computing; the flags and metadata that travel with every
// block of samples, Sec. 2.2).
//
// A flag covers one input over a block of L consecutive samples of a call.
// Flagged samples enter no visibility (they are replaced by the zero sample
// while the call's samples are copied into padded rows for the wide
// correlation kernel), and every pair counts the samples at which neither
// of its inputs was flagged:
//     n_ij = sum_b len_b * w_i(b) * w_j(b),   w = 1 - flag,
// kept per slot in int32 (n_ij <= T_MAX).  The counts come from bit-packed
// "unflagged" masks, 32 blocks per word: n_ij = L * popcount(w_i & w_j)
// over the full blocks, plus the last block's length if both are unflagged
// there.
//
// RFI excision: the spectral kurtosis of the M samples of each (block,
// input), from the power P = |x|^2 (Nita & Gary 2010),
//     SK = (M + 1) / (M - 1) * (M S2 / S1^2 - 1),  S1 = sum P, S2 = sum P^2,
// flagged when below lo or above hi (integer fractions over one
// denominator), or when S1 = 0.  The comparison is exact in 64-bit
// integers: with M <= 1024 and |P| <= 128, M S2 <= 2^34 and S1^2 <= 2^34, so
// both sides stay below 2^58 for thresholds up to 16.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

// Power sums of one byte (one complex sample) into s1, s2.
__device__ __forceinline__ void power_sums(uint32_t byte, int sh_re, int sh_im, int32_t &s1, int32_t &s2)
{
    const int re = (int)((byte >> sh_re) & 15u) - 8, im = (int)((byte >> sh_im) & 15u) - 8;
    const int p = re * re + im * im;
    s1 += p;
    s2 += p * p;
}

// The flag decision of one (block, input) from its sums over m samples.
__device__ __forceinline__ uint8_t sk_decide(int32_t s1, int32_t s2, int m, int64_t lo_num, int64_t hi_num,
                                             int64_t den)
{
    if (m < 2) return 0;
    if (s1 == 0) return 1;
    const int64_t a = s1, q = (int64_t)m * s2 - a * a;
    const int64_t num = (int64_t)(m + 1) * q, dd = (int64_t)(m - 1) * a * a;
    return (num * den < lo_num * dd || num * den > hi_num * dd) ? 1 : 0;
}

// Vector form: 16-byte-aligned rows with N % 16 == 0.  A workgroup takes
// 1024 inputs x one block: lane l of wave w loads the 16 inputs 16 l .. of
// rows w, w + 4, ... of the block (16-byte loads, a wave reading 1 KB
// contiguous per row), sums them, and the four waves' sums meet in LDS.
__global__ __launch_bounds__(256) void sk_flags_vec(const uint8_t *__restrict__ s, int64_t n_samples, int n,
                                                    int64_t stride, uint32_t re_low, int block_len, int64_t lo_num,
                                                    int64_t hi_num, int64_t den, uint8_t *__restrict__ flags)
{
    __shared__ int32_t red[4][1024][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = 1024 * (int)blockIdx.x + 16 * lane;
    const int64_t b = blockIdx.y;
    const int64_t t0 = b * block_len;
    const int64_t t1 = t0 + block_len < n_samples ? t0 + block_len : n_samples;
    const int sh_re = re_low ? 0 : 4, sh_im = re_low ? 4 : 0;
    int32_t s1[16], s2[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) s1[k] = s2[k] = 0;
    if (i0 < n) {
        const uint8_t *p = s + i0;
        int64_t t = t0 + wave;
        for (; t + 12 < t1; t += 16) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const uint4 *>(p + (t + 4 * u) * stride);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int k = 0; k < 16; ++k) power_sums((w4[k >> 2] >> (8 * (k & 3))) & 0xFFu, sh_re, sh_im, s1[k], s2[k]);
            }
        }
        for (; t < t1; t += 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p + t * stride);
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) power_sums((w4[k >> 2] >> (8 * (k & 3))) & 0xFFu, sh_re, sh_im, s1[k], s2[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        red[wave][16 * lane + k][0] = s1[k];
        red[wave][16 * lane + k][1] = s2[k];
    }
    __syncthreads();
    const int m = (int)(t1 - t0);
    for (int c = threadIdx.x; c < 1024; c += 256) {
        const int i = 1024 * (int)blockIdx.x + c;
        if (i >= n) continue;
        const int32_t a = red[0][c][0] + red[1][c][0] + red[2][c][0] + red[3][c][0];
        const int32_t q = red[0][c][1] + red[1][c][1] + red[2][c][1] + red[3][c][1];
        flags[b * n + i] = sk_decide(a, q, m, lo_num, hi_num, den);
    }
}

// Any alignment: one thread per (input, block), byte loads.
__global__ __launch_bounds__(256) void sk_flags_bytes(const uint8_t *__restrict__ s, int64_t n_samples, int n,
                                                      int64_t stride, uint32_t re_low, int block_len, int64_t lo_num,
                                                      int64_t hi_num, int64_t den, uint8_t *__restrict__ flags)
{
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    const int64_t b = blockIdx.y;
    if (i >= n) return;
    const int64_t t0 = b * block_len;
    const int64_t t1 = t0 + block_len < n_samples ? t0 + block_len : n_samples;
    const int sh_re = re_low ? 0 : 4, sh_im = re_low ? 4 : 0;
    int32_t s1 = 0, s2 = 0;
    for (int64_t t = t0; t < t1; ++t) power_sums(s[t * stride + i], sh_re, sh_im, s1, s2);
    flags[b * n + i] = sk_decide(s1, s2, (int)(t1 - t0), lo_num, hi_num, den);
}

// Rows of n samples copied into rows of n16 bytes, padded with the zero
// sample, every sample of a flagged (block, input) replaced by the zero
// sample.  Row t of the copy is sample t_first + t of the call, in block
// (t_first + t) / block_len.  Vector form (16-byte-aligned rows and flags,
// n % 16 == 0): a thread per 16 bytes, 16-byte loads of samples and flags,
// a workgroup covering 256 x 16 bytes of consecutive rows.
__device__ __forceinline__ uint32_t mask_word(uint32_t x, uint32_t f)
{
    // bytes of f that are nonzero -> 0xFF
    const uint32_t hi = ((f & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | f;
    const uint32_t m = ((hi >> 7) & 0x01010101u) * 0xFFu;
    return (x & ~m) | (0x88888888u & m);
}

__global__ __launch_bounds__(256) void mask_rows_vec(const uint8_t *__restrict__ src, int64_t stride, int n,
                                                     int64_t rows, uint8_t *__restrict__ dst,
                                                     const uint8_t *__restrict__ flags, int block_len,
                                                     int64_t t_first)
{
    const int per_row = n / 16;
    const int64_t total = rows * per_row;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t t = e / per_row;
        const int c = (int)(e - t * per_row) * 16;
        const uint4 x = *reinterpret_cast<const uint4 *>(src + t * stride + c);
        const uint4 f = *reinterpret_cast<const uint4 *>(flags + ((t_first + t) / block_len) * (int64_t)n + c);
        *reinterpret_cast<uint4 *>(dst + t * n + c) =
            make_uint4(mask_word(x.x, f.x), mask_word(x.y, f.y), mask_word(x.z, f.z), mask_word(x.w, f.w));
    }
}

// Any alignment or N: one workgroup per row, byte loads.
__global__ __launch_bounds__(256) void mask_rows(const uint8_t *__restrict__ src, int64_t stride, int n, int n16,
                                                 uint8_t *__restrict__ dst, const uint8_t *__restrict__ flags,
                                                 int block_len, int64_t t_first)
{
    const int64_t t = blockIdx.x;
    const uint8_t *row = src + t * stride;
    const uint8_t *frow = flags + ((t_first + t) / block_len) * (int64_t)n;
    uint32_t *out_row = reinterpret_cast<uint32_t *>(dst + t * n16);
    for (int c0 = 4 * (int)threadIdx.x; c0 < n16; c0 += 4 * 256) {
        uint32_t out = 0x88888888u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c0 + k;
            if (c < n && frow[c] == 0) out = (out & ~(0xFFu << (8 * k))) | ((uint32_t)row[c] << (8 * k));
        }
        out_row[c0 >> 2] = out;
    }
}

// Unflagged masks packed along blocks: bits[i][w] bit k set when block
// 32 w + k of input i is unflagged.  One wave per (two inputs, word): lane l
// reads block 32 w + l % 32 of input i0 + l / 32, and one ballot of the
// unflagged lanes holds both inputs' words.
__global__ __launch_bounds__(256) void pack_unflagged(const uint8_t *__restrict__ flags, int nb, int n, int words,
                                                      uint32_t *__restrict__ bits)
{
    const int lane = (int)threadIdx.x & 63;
    const int64_t wv = (int64_t)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const int64_t pairs = (n + 1) / 2;
    if (wv >= pairs * words) return;   // whole waves
    const int w = (int)(wv % words), i0 = 2 * (int)(wv / words);
    const int i = i0 + (lane >> 5), b = 32 * w + (lane & 31);
    const bool unflagged = i < n && b < nb && flags[(int64_t)b * n + i] == 0;
    const uint64_t m = __ballot(unflagged);
    if (lane == 0) bits[(int64_t)i0 * words + w] = (uint32_t)m;
    if (lane == 32 && i < n) bits[(int64_t)i * words + w] = (uint32_t)(m >> 32);
}

// Per-pair sample counts added into counts[k(i, j)] (packed upper triangle).
// A workgroup takes a 64 x 64 block of pairs (row block by, column block
// bx >= by); thread (ty, tx) takes rows 4 ty .. + 3 and columns tx + 16 q
// (q < 4), so that each row's 64 counts are updated by 16 consecutive
// threads at a time.  The masks of the 64 + 64 inputs go through LDS in
// chunks of up to CW words.  Blocks 0 .. nb-2 weigh block_len each, the
// last `last_len`.
constexpr int CW = 32;
__global__ __launch_bounds__(256) void count_pairs(const uint32_t *__restrict__ bits, int words, int nb, int n,
                                                   int block_len, int last_len, int32_t *__restrict__ counts)
{
    const int by = blockIdx.y, bx = blockIdx.x;
    if (bx < by) return;
    __shared__ uint32_t ra[64][CW + 1], cb[64][CW + 1];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    int32_t c[4][4] = {};
    const int last_w = (nb - 1) >> 5;
    const uint32_t last_bit = 1u << ((nb - 1) & 31);
    for (int w0 = 0; w0 < words; w0 += CW) {
        const int cw = words - w0 < CW ? words - w0 : CW;
        for (int e = tid; e < 64 * cw; e += 256) {
            const int r = e / cw, w = e % cw;
            const int ia = 64 * by + r, ib = 64 * bx + r;
            ra[r][w] = ia < n ? bits[(int64_t)ia * words + w0 + w] : 0u;
            cb[r][w] = ib < n ? bits[(int64_t)ib * words + w0 + w] : 0u;
        }
        __syncthreads();
        for (int w = 0; w < cw; ++w) {
            // the last block counts with its own length, below
            const uint32_t keep = (w0 + w == last_w) ? ~last_bit : 0xFFFFFFFFu;
            uint32_t a[4], b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                a[k] = ra[4 * ty + k][w] & keep;
                b[k] = cb[tx + 16 * k][w];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) c[p][q] += __popc(a[p] & b[q]);
        }
        __syncthreads();
    }
    bool lj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = 64 * bx + tx + 16 * q;
        lj[q] = j < n && (bits[(int64_t)j * words + last_w] & last_bit) != 0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int i = 64 * by + 4 * ty + p;
        if (i >= n) continue;
        const bool li = (bits[(int64_t)i * words + last_w] & last_bit) != 0;
        const int64_t row = (int64_t)i * n - (int64_t)i * (i - 1) / 2 - i;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 64 * bx + tx + 16 * q;
            if (j >= n || j < i) continue;
            counts[row + j] += c[p][q] * block_len + ((li && lj[q]) ? last_len : 0);
        }
    }
}

// out[k] = counts[k] + base (samples integrated without flags count for
// every pair).
__global__ __launch_bounds__(256) void counts_export(const int32_t *__restrict__ counts, int64_t npairs, int32_t base,
                                                     int32_t *__restrict__ out)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < npairs; k += (int64_t)gridDim.x * 256)
        out[k] = counts[k] + base;
}

hipError_t launch_sk_flags(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low,
                           int block_len, int64_t lo_num, int64_t hi_num, int64_t den, uint8_t *flags,
                           hipStream_t stream)
{
    const int64_t nb = (n_samples + block_len - 1) / block_len;
    if (nb <= 0) return hipSuccess;
    const bool vec = (reinterpret_cast<uintptr_t>(s) % 16) == 0 && stride % 16 == 0 && n % 16 == 0;
    if (vec)
        hipLaunchKernelGGL(sk_flags_vec, dim3((unsigned)((n + 1023) / 1024), (unsigned)nb), dim3(256), 0, stream, s,
                           n_samples, n, stride, re_low, block_len, lo_num, hi_num, den, flags);
    else
        hipLaunchKernelGGL(sk_flags_bytes, dim3((unsigned)((n + 255) / 256), (unsigned)nb), dim3(256), 0, stream, s,
                           n_samples, n, stride, re_low, block_len, lo_num, hi_num, den, flags);
    return hipGetLastError();
}

hipError_t launch_mask_rows(const uint8_t *src, int64_t stride, int n, int64_t rows, int n16, uint8_t *dst,
                            const uint8_t *flags, int block_len, int64_t t_first, hipStream_t stream)
{
    if (rows <= 0) return hipSuccess;
    const bool vec = n == n16 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 && stride % 16 == 0 &&
                     (reinterpret_cast<uintptr_t>(flags) % 16) == 0 && (reinterpret_cast<uintptr_t>(dst) % 16) == 0;
    if (vec) {
        int64_t blocks = (rows * (n / 16) + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(mask_rows_vec, dim3((unsigned)blocks), dim3(256), 0, stream, src, stride, n, rows, dst,
                           flags, block_len, t_first);
    } else {
        hipLaunchKernelGGL(mask_rows, dim3((unsigned)rows), dim3(256), 0, stream, src, stride, n, n16, dst, flags,
                           block_len, t_first);
    }
    return hipGetLastError();
}

hipError_t launch_counts(const uint8_t *flags, int nb, int n, int block_len, int last_len, uint32_t *bits,
                         int32_t *counts, hipStream_t stream)
{
    if (nb <= 0) return hipSuccess;
    const int words = (nb + 31) / 32;
    const int64_t waves = (int64_t)((n + 1) / 2) * words;   // one per (two inputs, word)
    hipLaunchKernelGGL(pack_unflagged, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, flags, nb, n, words,
                       bits);
    const unsigned tiles = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(count_pairs, dim3(tiles, tiles), dim3(256), 0, stream, bits, words, nb, n, block_len,
                       last_len, counts);
    return hipGetLastError();
}

hipError_t launch_counts_export(const int32_t *counts, int64_t npairs, int32_t base, int32_t *out,
                                hipStream_t stream)
{
    if (npairs <= 0) return hipSuccess;
    int64_t blocks = (npairs + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(counts_export, dim3((unsigned)blocks), dim3(256), 0, stream, counts, npairs, base, out);
    return hipGetLastError();
}

}  // namespace xeng
