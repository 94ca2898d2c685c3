// Phased-array beamforming (Sec. 2.1: the nodes form 10 phased-array beams
// for pulsar timing from the channelised samples; "Pulsar Beamforming" in
// Table tab:computing):
//     y_b(t) = sum_i w_bi x_i(t),
// complex int8 weights (parts in [-127, 127]) and 4+4-bit samples, exact
// int32 sums.  Per time sample this is a [1 x 2N] by [2N x 2B] real
// product, so a block of 16 time rows against up to 16 beams is one
// v_mfma_i32_16x16x64_i8 per 32 inputs and per output part:
//   A (rows = times)  : (Re x_i, Im x_i) pairs, 8 inputs per lane and step
//   B (cols = beams)  : (Re w, -Im w) pairs for Re y, (Im w, Re w) for Im y.
// The kernel reads every sample once, so it is bound by HBM bandwidth (about
// 10 complex MACs per sample byte for 10 beams), not by the matrix cores.
//
// Workgroup: 8 waves of 16 time rows (128 rows per row block), persistent
// over row blocks; the weights of up to 2048 inputs sit in LDS in operand
// order (64 B per input: 16 beams x 2 parts x 2 bytes), loaded once, or per
// chunk of 2048 inputs when N is larger.  A lane loads 16 bytes (16 inputs
// of its row) per pair of k-steps, eight pairs ahead of their MFMAs; the k
// index of a byte is (step, lane group, position), the same for A and B.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

typedef int bv4i __attribute__((ext_vector_type(4)));

constexpr int BEAM_CHUNK = 2048;                  // inputs whose weights fit in LDS
constexpr int BEAM_LDS = BEAM_CHUNK * 64;         // 128 KiB
constexpr int BEAMS_MAX = 16;
constexpr int BEAM_WAVES = 8;                     // waves per workgroup, 16 time rows each

// Interleave the offset-decoded nibbles of 4 packed samples into (re, im)
// int8 pairs: two dwords [re0 im0 re1 im1], [re2 im2 re3 im3].
__device__ __forceinline__ void unpack4(uint32_t w, bool re_low, uint32_t &o0, uint32_t &o1)
{
    const uint32_t hi = (((w >> 4) & 0x0F0F0F0Fu) + 0x78787878u) ^ 0x80808080u;   // nibble - 8
    const uint32_t lo = ((w & 0x0F0F0F0Fu) + 0x78787878u) ^ 0x80808080u;
    const uint32_t re = re_low ? lo : hi, im = re_low ? hi : lo;
    // v_perm selector bytes: 0-3 pick from the second source, 4-7 from the first
    o0 = __builtin_amdgcn_perm(im, re, 0x05010400u);   // re0 im0 re1 im1
    o1 = __builtin_amdgcn_perm(im, re, 0x07030602u);   // re2 im2 re3 im3
}

// The weights of one chunk of BEAM_CHUNK inputs, already in operand order
// in device memory (arranged on the host, see xeng_beams_create), into LDS:
// 16-byte loads, all issued before any store.
__device__ __forceinline__ void load_weights(uint8_t *lw, const uint4 *__restrict__ w)
{
    constexpr int PER = BEAM_LDS / 16 / (64 * BEAM_WAVES);
    uint4 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = w[threadIdx.x + k * blockDim.x];
#pragma unroll
    for (int k = 0; k < PER; ++k) reinterpret_cast<uint4 *>(lw)[threadIdx.x + k * blockDim.x] = v[k];
}

// 16 inputs i0 .. of a row (the zero sample where out of range).
template <bool VEC>
__device__ __forceinline__ uint4 load16(const uint8_t *row, bool row_ok, int i0, int cn)
{
    uint4 v = make_uint4(0x88888888u, 0x88888888u, 0x88888888u, 0x88888888u);
    if (!row_ok || i0 >= cn) return v;
    if (VEC) return *reinterpret_cast<const uint4 *>(row + i0);
    uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (i0 + k < cn) x[k >> 2] = (x[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | ((uint32_t)row[i0 + k] << (8 * (k & 3)));
    return make_uint4(x[0], x[1], x[2], x[3]);
}

// Two k-steps (16 inputs of the lane's row) into both accumulators.
__device__ __forceinline__ void beam_steps(bv4i &acc_re, bv4i &acc_im, const uint4 x, const uint8_t *lw, int p,
                                           int g, int r, bool re_low)
{
    const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint32_t a[4];
        unpack4(xs[2 * h], re_low, a[0], a[1]);
        unpack4(xs[2 * h + 1], re_low, a[2], a[3]);
        const bv4i av = {(int)a[0], (int)a[1], (int)a[2], (int)a[3]};
        const int off = (((2 * p + h) * 4 + g) * 16 + r) * 16;
        const bv4i br = *reinterpret_cast<const bv4i *>(lw + off);
        const bv4i bi = *reinterpret_cast<const bv4i *>(lw + BEAM_LDS / 2 + off);
        acc_re = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, br, acc_re, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bi, acc_im, 0, 0, 0);
    }
}

// Loads run PREF pairs of k-steps ahead of the MFMAs that use them
// (register double buffer), so that each wave keeps PREF KiB of samples in
// flight.
constexpr int PREF = 8;

template <bool VEC, bool QUANT>
__global__ __launch_bounds__(64 * BEAM_WAVES, 1) void beamform(const uint8_t *__restrict__ s, int64_t n_samples,
                                                               int n, int64_t stride, uint32_t re_low,
                                                               const int8_t *__restrict__ w, int n_beams, int shift,
                                                               void *__restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lw[];   // [re part | im part], BEAM_LDS / 2 each
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    constexpr int ROWS = 16 * BEAM_WAVES;
    const int64_t row_blocks = (n_samples + ROWS - 1) / ROWS;
    const bool one_chunk = n <= BEAM_CHUNK;
    const uint4 *wc = reinterpret_cast<const uint4 *>(w);
    if (one_chunk) {
        load_weights(lw, wc);
        __syncthreads();
    }
    for (int64_t rb = blockIdx.x; rb < row_blocks; rb += gridDim.x) {
        const int64_t t = rb * ROWS + wave * 16 + r;     // this lane's time row
        const bool row_ok = t < n_samples;
        bv4i acc_re = {0, 0, 0, 0}, acc_im = {0, 0, 0, 0};
        for (int c0 = 0; c0 < n; c0 += BEAM_CHUNK) {
            const int cn = min(BEAM_CHUNK, n - c0);
            const int np = (cn + 63) / 64;               // pairs of k-steps
            if (!one_chunk) {
                __syncthreads();
                load_weights(lw, wc + (int64_t)(c0 / BEAM_CHUNK) * (BEAM_LDS / 16));
                __syncthreads();
            }
            const uint8_t *row = s + (row_ok ? t : 0) * stride + c0;
            uint4 cur[PREF], nxt[PREF];
#pragma unroll
            for (int k = 0; k < PREF; ++k) cur[k] = load16<VEC>(row, row_ok && k < np, 64 * k + 16 * g, cn);
            for (int p0 = 0; p0 < np; p0 += PREF) {
#pragma unroll
                for (int k = 0; k < PREF; ++k)
                    nxt[k] = load16<VEC>(row, row_ok && p0 + PREF + k < np, 64 * (p0 + PREF + k) + 16 * g, cn);
#pragma unroll
                for (int k = 0; k < PREF; ++k)
                    if (p0 + k < np) beam_steps(acc_re, acc_im, cur[k], lw, p0 + k, g, r, re_low != 0);
#pragma unroll
                for (int k = 0; k < PREF; ++k) cur[k] = nxt[k];
            }
        }
        // C of a 16 x 16 block: lane holds column (beam) lane % 16, rows
        // 4 (lane / 16) .. + 3 of the wave's 16 time rows
        const int b = lane & 15;
        if (b < n_beams) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t tt = rb * ROWS + wave * 16 + 4 * g + k;
                if (tt >= n_samples) continue;
                const int64_t o = (tt * n_beams + b) * 2;
                if (QUANT) {
                    // divide by 2^shift, rounded half to even, clipped to [-127, 127]
                    int32_t v2[2] = {acc_re[k], acc_im[k]};
                    int8_t q[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        int64_t v = v2[u];
                        if (shift > 0) v = (v + (INT64_C(1) << (shift - 1)) - 1 + ((v >> shift) & 1)) >> shift;
                        q[u] = (int8_t)(v < -127 ? -127 : (v > 127 ? 127 : v));
                    }
                    int8_t *po = reinterpret_cast<int8_t *>(out) + o;
                    po[0] = q[0];
                    po[1] = q[1];
                } else {
                    int32_t *po = reinterpret_cast<int32_t *>(out) + o;
                    po[0] = acc_re[k];
                    po[1] = acc_im[k];
                }
            }
        }
    }
}

// Operand-order image of the weights (host): nchunks x BEAM_LDS bytes, the
// LDS contents of each chunk of BEAM_CHUNK inputs as the kernel expects them.
// Input i of a chunk, beam b: step s = 2 (i / 64) + (i % 16) / 8, lane group
// (i % 64) / 16; byte offset ((4 s + group) * 16 + b) * 16 + 2 (i % 8) holds
// (Re w, -Im w) in the first half of the image (Re y) and (Im w, Re w) in
// the second (Im y).  Inputs past N and beams past n_beams are zero.
int64_t beam_image_bytes(int n) { return (int64_t)((n + BEAM_CHUNK - 1) / BEAM_CHUNK) * BEAM_LDS; }

void beam_image(const int8_t *w, int n, int n_beams, uint8_t *img)
{
    const int nchunks = (n + BEAM_CHUNK - 1) / BEAM_CHUNK;
    for (int c = 0; c < nchunks; ++c) {
        uint8_t *re = img + (int64_t)c * BEAM_LDS, *im = re + BEAM_LDS / 2;
        for (int i = 0; i < BEAM_CHUNK; ++i) {
            const int gi = c * BEAM_CHUNK + i;
            const int step = 2 * (i / 64) + (i % 16) / 8, grp = (i % 64) / 16;
            for (int b = 0; b < BEAMS_MAX; ++b) {
                int wr = 0, wi = 0;
                if (gi < n && b < n_beams) {
                    wr = w[((int64_t)b * n + gi) * 2];
                    wi = w[((int64_t)b * n + gi) * 2 + 1];
                }
                const int off = ((step * 4 + grp) * 16 + b) * 16 + 2 * (i % 8);
                re[off] = (uint8_t)(int8_t)wr;
                re[off + 1] = (uint8_t)(int8_t)(-wi);
                im[off] = (uint8_t)(int8_t)wi;
                im[off + 1] = (uint8_t)(int8_t)wr;
            }
        }
    }
}

hipError_t init_beam_kernel()
{
    hipError_t e = hipFuncSetAttribute((const void *)beamform<true, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, BEAM_LDS);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)beamform<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                BEAM_LDS);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)beamform<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                BEAM_LDS);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)beamform<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                BEAM_LDS);
    return e;
}

hipError_t launch_beamform(const uint8_t *s, int64_t n_samples, int n, int64_t stride, uint32_t re_low,
                           const int8_t *d_w, int n_beams, int shift, void *out, int grid, hipStream_t stream)
{
    if (n_samples <= 0) return hipSuccess;
    const bool vec = (reinterpret_cast<uintptr_t>(s) % 16) == 0 && stride % 16 == 0 && n % 16 == 0;
    const bool quant = shift >= 0;
    const dim3 g((unsigned)grid), b(64 * BEAM_WAVES);
    if (vec && quant)
        hipLaunchKernelGGL((beamform<true, true>), g, b, BEAM_LDS, stream, s, n_samples, n, stride, re_low, d_w,
                           n_beams, shift, out);
    else if (vec)
        hipLaunchKernelGGL((beamform<true, false>), g, b, BEAM_LDS, stream, s, n_samples, n, stride, re_low, d_w,
                           n_beams, shift, out);
    else if (quant)
        hipLaunchKernelGGL((beamform<false, true>), g, b, BEAM_LDS, stream, s, n_samples, n, stride, re_low, d_w,
                           n_beams, shift, out);
    else
        hipLaunchKernelGGL((beamform<false, false>), g, b, BEAM_LDS, stream, s, n_samples, n, stride, re_low, d_w,
                           n_beams, shift, out);
    return hipGetLastError();
}

}  // namespace xeng
