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
//   Re V = [Re x_i | Im x_i] . [Re x_j | Im x_j]   = Re_i Re_j + Im_i Im_j
//   Im V = [Im x_i | -Re x_i] . [Re x_j | Im x_j]  = Im_i Re_j - Re_i Im_j
// so the row (A) side keeps three int8 vectors per sample group (Re, Im,
// -Re) and the column (B) side two (Re, Im); one B operand feeds both
// products.  Every partial sum is an exact int32.
//
// Data path per 32-sample stage (double-buffered in LDS):
//   global (time-major bytes) -> dword loads, 4 inputs x 8 samples per lane
//   -> 4x4 byte transposes (v_perm) -> nibble unpack to int8 -> LDS
//   -> ds_read_b128 operands -> v_mfma_i32_32x32x32_i8.
// The paper's own design packed several low-bit products into 24-bit
// multiply-adds on GCN3 (Sec. 2.3, "GPUs"); on CDNA4 the int8 matrix cores
// do this work instead (Sec. 4.1 anticipates low-bit matrix units).
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// LDS stage layout.  For each k-step q (16 samples) a component region holds
// 128 tile positions x 16 bytes (the 16 samples of one input, in time
// order).  A rows keep Re, Im, -Re; B rows keep Re, Im.  Position p of a
// tile row offset r is 32*(r % 4) + r/4, so that the staging writes of a
// wave land on consecutive 16-byte slots (no bank conflicts) while the MFMA
// operand reads stay contiguous too.
constexpr int CH = TILE * 16;       // 2048 bytes
constexpr int A_Q = 3 * CH;
constexpr int B_Q = 2 * CH;
constexpr int A_BYTES = 2 * A_Q;    // 2 k-steps per stage
constexpr int B_BYTES = 2 * B_Q;
constexpr int STAGE_BYTES = A_BYTES + B_BYTES;   // 20480

__device__ __forceinline__ uint32_t vperm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    return __builtin_amdgcn_perm(s0, s1, sel);
}

// 4 x 4 byte transpose: rows a, b, c, d are 4 inputs at 4 consecutive times;
// out[k] holds input k at the 4 times (byte = time).
__device__ __forceinline__ void transpose4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                           uint32_t out[4])
{
    const uint32_t ab_lo = vperm(b, a, 0x05010400u);   // a0 b0 a1 b1
    const uint32_t ab_hi = vperm(b, a, 0x07030602u);   // a2 b2 a3 b3
    const uint32_t cd_lo = vperm(d, c, 0x05010400u);
    const uint32_t cd_hi = vperm(d, c, 0x07030602u);
    out[0] = vperm(cd_lo, ab_lo, 0x05040100u);         // a0 b0 c0 d0
    out[1] = vperm(cd_lo, ab_lo, 0x07060302u);         // a1 b1 c1 d1
    out[2] = vperm(cd_hi, ab_hi, 0x05040100u);
    out[3] = vperm(cd_hi, ab_hi, 0x07060302u);
}

// Offset-binary nibbles (0..15, one per byte) -> signed int8 value and its
// negation, four at a time, with no carries between bytes:
//   n - 8 = (n + 0x78) ^ 0x80,   8 - n = (0x88 - n) ^ 0x80.
__device__ __forceinline__ uint32_t nib_to_i8(uint32_t n) { return (n + 0x78787878u) ^ 0x80808080u; }
__device__ __forceinline__ uint32_t nib_to_neg_i8(uint32_t n) { return (0x88888888u - n) ^ 0x80808080u; }

// Load the 4 inputs [i0, i0+4) of one lane for 8 consecutive samples
// starting at t_first; samples at or past t1 and inputs past n read as the
// zero sample 0x88.
__device__ __forceinline__ void stage_load(uint32_t d[8], const uint8_t *col, int64_t stride,
                                           int t_first, int t1, bool fast, int nvalid)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int t = t_first + k;
        const int tc = t < t1 ? t : t1 - 1;
        const uint8_t *p = col + (int64_t)tc * stride;
        uint32_t v;
        if (fast) {
            v = *(const uint32_t *)p;
        } else {
            v = 0x88888888u;
            for (int b = 0; b < nvalid; ++b)
                v = (v & ~(0xFFu << (8 * b))) | ((uint32_t)p[b] << (8 * b));
        }
        d[k] = t < t1 ? v : 0x88888888u;
    }
}

// Transpose + unpack one lane's 4 inputs x 8 samples into the stage buffer.
__device__ __forceinline__ void stage_write(uint8_t *region, const uint32_t d[8], int g, int hl,
                                            bool role_a, bool re_low)
{
    uint32_t p0[4], p1[4];
    transpose4(d[0], d[1], d[2], d[3], p0);
    transpose4(d[4], d[5], d[6], d[7], p1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t h0 = (p0[c] >> 4) & 0x0F0F0F0Fu, l0 = p0[c] & 0x0F0F0F0Fu;
        const uint32_t h1 = (p1[c] >> 4) & 0x0F0F0F0Fu, l1 = p1[c] & 0x0F0F0F0Fu;
        const uint32_t re0 = re_low ? l0 : h0, im0 = re_low ? h0 : l0;
        const uint32_t re1 = re_low ? l1 : h1, im1 = re_low ? h1 : l1;
        const int off = 16 * (32 * c + g) + 8 * hl;
        *(uint2 *)(region + off) = make_uint2(nib_to_i8(re0), nib_to_i8(re1));
        *(uint2 *)(region + CH + off) = make_uint2(nib_to_i8(im0), nib_to_i8(im1));
        if (role_a)
            *(uint2 *)(region + 2 * CH + off) = make_uint2(nib_to_neg_i8(re0), nib_to_neg_i8(re1));
    }
}

__device__ __forceinline__ v4i lds128(const uint8_t *p) { return *(const v4i *)p; }

__device__ __forceinline__ void flush_block(int32_t *blk, const v16i &re, const v16i &im,
                                            bool atomic)
{
    if (atomic) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            __hip_atomic_fetch_add(blk + r * 64, re[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(blk + 1024 + r * 64, im[r], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            blk[r * 64] += re[r];
            blk[1024 + r * 64] += im[r];
        }
    }
}

// Persistent correlation kernel: workgroup w runs pieces [wg_off[w], wg_off[w+1]).
// 256 threads = 4 waves; wave (wa, wb) owns MFMA blocks ca in {2wa, 2wa+1},
// cb in {2wb, 2wb+1} of the tile (64 x 64 outputs, Re and Im).
__global__ __launch_bounds__(256, 2) void xcorr_mfma(KernelArgs args)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * STAGE_BYTES];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wb = wave & 1;
    // staging role of this lane: input group g (4 inputs), half hl of a
    // k-step, k-step q_st of the stage, A rows (waves 0, 1) or B rows (2, 3)
    const int g = (lane & 7) + 8 * (lane >> 4);
    const int hl = (lane >> 3) & 1;
    const int q_st = wave & 1;
    const bool role_a = wave < 2;

    const int p_begin = args.wg_off[blockIdx.x], p_end = args.wg_off[blockIdx.x + 1];
    for (int pi = p_begin; pi < p_end; ++pi) {
        const Piece pc = args.pieces[pi];
        const JobDesc jd = args.jobs ? args.jobs[pc.job] : args.job0;
        const int ti = pc.tile & 0xFFFF, tj = (pc.tile >> 16) & 0xFFFF;
        const bool diag = ti == tj;
        const int t0 = pc.t0;
        const int t1 = pc.t1_atomic & 0x7FFFFFFF;
        const bool atomic = pc.t1_atomic < 0;
        const bool re_low = (jd.flags & JOB_RE_LOW) != 0;

        // this lane's staging source: 4 inputs of the A (ti) or B (tj) block
        const bool stager = role_a || !diag;
        const int i0 = (role_a ? ti : tj) * TILE + 4 * g;
        const int nvalid = min(max(jd.n - i0, 0), 4);
        const bool fast = (jd.flags & JOB_ALIGNED4) && nvalid == 4;
        const uint8_t *col = jd.samples + (nvalid > 0 ? i0 : 0);
        const int t_lane = 16 * q_st + 8 * hl;     // first sample of this lane in a stage

        v16i acc_re[2][2], acc_im[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc_re[a][b][r] = 0;
                    acc_im[a][b][r] = 0;
                }

        const int nst = (t1 - t0 + STAGE - 1) / STAGE;
        uint32_t d[8];
        if (stager) {
            if (nvalid > 0) stage_load(d, col, jd.stride, t0 + t_lane, t1, fast, nvalid);
            else for (int k = 0; k < 8; ++k) d[k] = 0x88888888u;
            uint8_t *region = smem + (role_a ? q_st * A_Q : A_BYTES + q_st * B_Q);
            stage_write(region, d, g, hl, role_a, re_low);
        }
        __syncthreads();

        for (int s = 0; s < nst; ++s) {
            const bool more = s + 1 < nst;
            if (more && stager && nvalid > 0)
                stage_load(d, col, jd.stride, t0 + (s + 1) * STAGE + t_lane, t1, fast, nvalid);

            const uint8_t *buf = smem + (s & 1) * STAGE_BYTES;
            const uint8_t *bbuf = diag ? buf : buf + A_BYTES;
            const int bq = diag ? A_Q : B_Q;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint8_t *aq = buf + q * A_Q + (lane >> 5) * CH + 16 * (lane & 31);
                const v4i re_a0 = lds128(aq + 512 * (2 * wa));
                const v4i re_a1 = lds128(aq + 512 * (2 * wa + 1));
                const v4i im_a0 = lds128(aq + CH + 512 * (2 * wa));
                const v4i im_a1 = lds128(aq + CH + 512 * (2 * wa + 1));
                const uint8_t *bp = bbuf + q * bq + (lane >> 5) * CH + 16 * (lane & 31);
                const v4i b0 = lds128(bp + 512 * (2 * wb));
                const v4i b1 = lds128(bp + 512 * (2 * wb + 1));
                acc_re[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a0, b0, acc_re[0][0], 0, 0, 0);
                acc_im[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a0, b0, acc_im[0][0], 0, 0, 0);
                acc_re[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a0, b1, acc_re[0][1], 0, 0, 0);
                acc_im[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a0, b1, acc_im[0][1], 0, 0, 0);
                acc_re[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a1, b0, acc_re[1][0], 0, 0, 0);
                acc_im[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a1, b0, acc_im[1][0], 0, 0, 0);
                acc_re[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(re_a1, b1, acc_re[1][1], 0, 0, 0);
                acc_im[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im_a1, b1, acc_im[1][1], 0, 0, 0);
            }

            if (more && stager) {
                if (nvalid == 0)
                    for (int k = 0; k < 8; ++k) d[k] = 0x88888888u;
                uint8_t *region = smem + ((s + 1) & 1) * STAGE_BYTES +
                                  (role_a ? q_st * A_Q : A_BYTES + q_st * B_Q);
                stage_write(region, d, g, hl, role_a, re_low);
            }
            __syncthreads();
        }

        // integrate into the slot's accumulators
        const int64_t tile_idx = (int64_t)ti * jd.nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
        int32_t *tb = jd.acc + tile_idx * TILE_I32 + lane;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                flush_block(tb + ((2 * wa + a) * BLKS + (2 * wb + b)) * BLOCK_I32,
                            acc_re[a][b], acc_im[a][b], atomic);
    }
}

// Accumulators (tile layout) -> packed row-major upper triangle of (Re, Im).
__global__ __launch_bounds__(256) void vis_dump(const int32_t *__restrict__ acc, int n, int nt,
                                                int32_t *__restrict__ out)
{
    const int i = blockIdx.y;
    const int j = i + blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int ti = i >> 7, tj = j >> 7;
    const int ri = i & 127, rj = j & 127;
    const int pa = 32 * (ri & 3) + (ri >> 2), pb = 32 * (rj & 3) + (rj >> 2);
    const int ca = pa >> 5, ra = pa & 31, cb = pb >> 5, lb = pb & 31;
    const int reg = 4 * (ra >> 3) + (ra & 3);
    const int ln = lb + 32 * ((ra >> 2) & 1);
    const int64_t tile = (int64_t)ti * nt - (int64_t)ti * (ti - 1) / 2 + (tj - ti);
    const int32_t *p = acc + tile * TILE_I32 + (ca * BLKS + cb) * BLOCK_I32 + reg * 64 + ln;
    const int64_t k = (int64_t)i * n - (int64_t)i * (i - 1) / 2 + (j - i);
    reinterpret_cast<int2 *>(out)[k] = make_int2(p[0], p[1024]);
}

__global__ __launch_bounds__(256) void fill_zero(int4 *__restrict__ p, int64_t n4)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n4;
         k += (int64_t)gridDim.x * 256)
        p[k] = make_int4(0, 0, 0, 0);
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
hipError_t launch_correlate(const KernelArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(xcorr_mfma, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_dump(const int32_t *acc, int n, int nt, int32_t *out, hipStream_t stream)
{
    dim3 grid((n + 255) / 256, n);
    hipLaunchKernelGGL(vis_dump, grid, dim3(256), 0, stream, acc, n, nt, out);
    return hipGetLastError();
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
