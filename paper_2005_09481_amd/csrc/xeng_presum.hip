// The unsigned-nibble form with O(N) pre-sums (xeng_correlate_presum): the
// paper's GPUs multiplied the stored 4-bit values and corrected the result
// with O(N) bookkeeping (Sec. 2.3, "GPUs"; Table tab:computing, "Re-Order and
// Pre-Sum").  With u = x + 8 and, per input, SR = sum_t uR, SI = sum_t uI
// over the call's T samples:
//   Re V_ij = U_re - 8 (SR_i + SI_i + SR_j + SI_j) + 128 T
//   Im V_ij = U_im + 8 (SR_i - SI_i) - 8 (SR_j - SI_j)
// where U are the sums of unsigned products the UNSIGNED instances of the
// general kernel add into the slot.  presum_cols forms SR and SI; the
// correction kernel then adds, to every pair i <= j < N of the slot, the
// terms above -- in the slot's stored form, whose imaginary part is
// Im V_ij - S_j with S_j = sum_t Im x_j = SI_j - 8 T.  The slot words are
// 64-bit (Im 2^32 + Re) sums, exact in modular arithmetic, so the unsigned
// sums may pass the int32 range before the correction brings every pair
// back to its exact value.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

// Column sums of the nibbles: workgroup (x, y) takes inputs 256 x .. of
// rows y, y + gridDim.y, ...; atomic adds of its partial sums into sr, si
// (zeroed before).
__global__ __launch_bounds__(256) void presum_cols(const uint8_t *__restrict__ s, int64_t n_samples, int n,
                                                   int64_t stride, uint32_t re_low, int32_t *__restrict__ sr,
                                                   int32_t *__restrict__ si)
{
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i >= n) return;
    int32_t a = 0, b = 0;
    for (int64_t t = blockIdx.y; t < n_samples; t += gridDim.y) {
        const uint32_t v = s[t * stride + i];
        a += (int32_t)(v >> 4);
        b += (int32_t)(v & 15u);
    }
    atomicAdd(sr + i, re_low ? b : a);
    atomicAdd(si + i, re_low ? a : b);
}

// Thread per 64-bit word of the slot's tile layout (tile-major over the
// upper triangle of tiles; in a tile [ca][cb][reg][lane], row 8 (reg / 4) +
// 4 (lane / 32) + reg % 4 of block ca, column lane % 32 of block cb).
// Workgroup (x, y): tile row ti = y, tile column ti + x / 64, words
// 256 (x % 64) .. of that tile.
__global__ __launch_bounds__(256) void presum_correct(uint64_t *__restrict__ acc, int n, int nt, int64_t n_samples,
                                                      const int32_t *__restrict__ sr, const int32_t *__restrict__ si)
{
    const int ti = blockIdx.y, tj = ti + (int)(blockIdx.x / 64);
    if (tj >= nt) return;
    const int w = (int)(blockIdx.x % 64) * 256 + (int)threadIdx.x;
    const int64_t tile = (int64_t)ti * nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
    const int blk = w / (int)BLOCK_W, ca = blk / BLKS, cb = blk % BLKS;
    const int rl = w % (int)BLOCK_W, reg = rl / 64, lane = rl % 64;
    const int i = TILE * ti + BLK * ca + 8 * (reg / 4) + 4 * (lane / 32) + reg % 4;
    const int j = TILE * tj + BLK * cb + lane % 32;
    if (i > j || j >= n) return;
    const int64_t t = n_samples;
    const int64_t ri = sr[i], ii = si[i], rj = sr[j], ij = si[j];
    const int64_t d_re = -8 * (ri + ii + rj + ij) + 128 * t;
    const int64_t d_im = 8 * (ri - ii) - 8 * (rj - ij) - (ij - 8 * t);
    acc[tile * TILE_W + w] += ((uint64_t)d_im << 32) + (uint64_t)d_re;
}

hipError_t launch_presum(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low, int32_t *sr,
                         int32_t *si, hipStream_t stream)
{
    if (n_samples <= 0) return hipSuccess;
    int64_t rows = n_samples < 256 ? n_samples : 256;
    hipLaunchKernelGGL(presum_cols, dim3((unsigned)((n + 255) / 256), (unsigned)rows), dim3(256), 0, stream, s,
                       n_samples, n, stride, re_low, sr, si);
    return hipGetLastError();
}

hipError_t launch_presum_correct(int32_t *acc, int n, int nt, int64_t n_samples, const int32_t *sr,
                                 const int32_t *si, hipStream_t stream)
{
    static_assert(TILE_W == 64 * 256, "64 workgroups of 256 words per tile");
    hipLaunchKernelGGL(presum_correct, dim3((unsigned)(64 * nt), (unsigned)nt), dim3(256), 0, stream,
                       reinterpret_cast<uint64_t *>(acc), n, nt, n_samples, sr, si);
    return hipGetLastError();
}

}  // namespace xeng
