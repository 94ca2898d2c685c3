// The unsigned-nibble form with O(N) pre-sums (xeng_correlate_presum): the
// paper's GPUs multiplied the stored 4-bit values and corrected the result
// with O(N) bookkeeping (Sec. 2.3, "GPUs"; Table tab:computing, "Re-Order and
// Pre-Sum").  With u = x + 8 and, per input, SR = sum_t uR, SI = sum_t uI
// over the call's T samples:
//   Re V_ij = U_re - 8 (SR_i + SI_i + SR_j + SI_j) + 128 T
//   Im V_ij = U_im + 8 (SR_i - SI_i) - 8 (SR_j - SI_j)
// where U are the sums of unsigned products the unsigned instances of the
// correlation kernels add into the slot.  presum_cols (presum_cols16 for
// aligned rows) forms SR and SI; the
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

// The same sums for 16-byte rows at a 16-byte-aligned base with N a multiple
// of 16 (the arrays the wide kernel reads in place).  A workgroup takes 256
// inputs (16 column groups of 16 bytes) of a slice of rows_per_wg rows,
// its 16 row lanes reading every 16th row of it with one 16-byte load each,
// all of a lane's loads for 16 rows in flight together.  Nibbles add in byte
// lanes (16 rows of at most 15 fit a byte) before they widen into the 32
// per-input sums; the row lanes then meet in LDS and one atomic add per
// input and sum leaves the workgroup.
constexpr int PS_LANES = 16;    // row lanes per workgroup
constexpr int PS_GROUPS = 16;   // 16-byte column groups per workgroup
constexpr int PS_ROWS = 16;     // rows per lane between widenings
typedef unsigned int pv4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void presum_cols16(const uint8_t *__restrict__ s, int64_t n_samples, int n,
                                                     int64_t stride, int64_t rows_per_wg, uint32_t re_low,
                                                     int32_t *__restrict__ sr, int32_t *__restrict__ si)
{
    __shared__ int32_t part[2][PS_LANES][PS_GROUPS * 16];   // 32 KiB: high, low nibble sums per lane
    const int g = (int)threadIdx.x % PS_GROUPS, r = (int)threadIdx.x / PS_GROUPS;
    const int col = ((int)blockIdx.x * PS_GROUPS + g) * 16;
    const int64_t t0 = (int64_t)blockIdx.y * rows_per_wg;
    const int64_t t1 = t0 + rows_per_wg < n_samples ? t0 + rows_per_wg : n_samples;
    int32_t hi[16], lo[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) hi[k] = lo[k] = 0;
    if (col < n) {
        const uint8_t *p = s + col;
        for (int64_t tb = t0 + r; tb < t1; tb += (int64_t)PS_LANES * PS_ROWS) {
            pv4u v[PS_ROWS];
#pragma unroll
            for (int k = 0; k < PS_ROWS; ++k) {
                const int64_t t = tb + (int64_t)PS_LANES * k;
                v[k] = t < t1 ? *reinterpret_cast<const pv4u *>(p + t * stride) : pv4u{0u, 0u, 0u, 0u};
            }
            pv4u bl = {0u, 0u, 0u, 0u}, bh = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int k = 0; k < PS_ROWS; ++k) {
                bl += v[k] & 0x0F0F0F0Fu;
                bh += (v[k] >> 4u) & 0x0F0F0F0Fu;
            }
#pragma unroll
            for (int w = 0; w < 4; ++w)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    lo[4 * w + b] += (int32_t)((bl[w] >> (8 * b)) & 255u);
                    hi[4 * w + b] += (int32_t)((bh[w] >> (8 * b)) & 255u);
                }
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        part[0][r][g * 16 + k] = hi[k];
        part[1][r][g * 16 + k] = lo[k];
    }
    __syncthreads();
    const int i = (int)blockIdx.x * PS_GROUPS * 16 + (int)threadIdx.x;
    if (i >= n) return;
    int32_t a = 0, b = 0;
#pragma unroll
    for (int q = 0; q < PS_LANES; ++q) {
        a += part[0][q][threadIdx.x];
        b += part[1][q][threadIdx.x];
    }
    atomicAdd(sr + i, re_low ? b : a);
    atomicAdd(si + i, re_low ? a : b);
}

hipError_t launch_presum(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low, int32_t *sr,
                         int32_t *si, hipStream_t stream)
{
    if (n_samples <= 0) return hipSuccess;
    static_assert(PS_LANES * PS_GROUPS == 256, "one thread per row lane and column group");
    if (reinterpret_cast<uintptr_t>(s) % 16 == 0 && stride % 16 == 0 && n % 16 == 0) {
        // about 1024 workgroups, whole blocks of 16 rows per lane
        const int64_t gx = (n + 255) / 256;
        const int64_t block = (int64_t)PS_LANES * PS_ROWS;
        const int64_t gy_want = 1024 / gx > 1 ? 1024 / gx : 1;
        int64_t rows = (n_samples + gy_want - 1) / gy_want;
        rows = (rows + block - 1) / block * block;
        const int64_t gy = (n_samples + rows - 1) / rows;
        hipLaunchKernelGGL(presum_cols16, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, stream, s, n_samples, n,
                           stride, rows, re_low, sr, si);
        return hipGetLastError();
    }
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
