// Measurement only: the int8 matrix-core rate a device sustains under its
// power limit.  Every CU runs a loop of nothing but v_mfma_i32_32x32x32_i8
// in the correlation kernel's shape -- eight waves, two per SIMD, eight
// independent accumulators of a 32 x 32 block per wave -- on operands of the
// form the correlation kernels feed the matrix cores (bytes 16 x a 4-bit
// value), four operand sets per wave used in turn, so that every
// instruction's operands differ from the previous one's as a correlator's
// do.  No memory traffic, no LDS, no other instructions in the loop: the
// rate it reaches bounds every int8 kernel on the part at the clock the part
// holds under that load.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"

namespace xeng {

typedef int cv4i __attribute__((ext_vector_type(4)));
typedef int cv16i __attribute__((ext_vector_type(16)));

constexpr int CEIL_WAVES = 8;
constexpr int CEIL_ACC = 8;

// A 32-bit mixing step (the finaliser of a multiplicative hash) for operand
// bytes that differ by lane, wave, workgroup and operand set.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// clk (workgroup 0): shader-clock cycles and 100 MHz time at the start
// ([0], [1]) when stamp_start, at the end ([2], [3]) when stamp_end.
__global__ __launch_bounds__(64 * CEIL_WAVES, 1) void mfma_ceiling(int iters, int32_t *__restrict__ out,
                                                                    int64_t *__restrict__ clk, int stamp_start,
                                                                    int stamp_end)
{
    const bool stamp = blockIdx.x == 0 && threadIdx.x == 0;
    if (stamp && stamp_start) {
        clk[0] = (int64_t)__builtin_amdgcn_s_memtime();
        clk[1] = (int64_t)__builtin_amdgcn_s_memrealtime();
    }
    const uint32_t seed = (blockIdx.x * 64u * CEIL_WAVES + threadIdx.x) * 0x9E3779B9u;
    cv4i a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[k][j] = (int)(mix32(seed + 8u * k + j) & 0xF0F0F0F0u);
            b[k][j] = (int)(mix32(seed + 8u * k + j + 4u) & 0xF0F0F0F0u);
        }
    cv16i acc[CEIL_ACC];
#pragma unroll
    for (int k = 0; k < CEIL_ACC; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0;
    // four rounds per trip, so that every operand index is a constant; the
    // sums wrap (int32), which changes nothing here
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < CEIL_ACC; ++k)
                acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[(k + u) & 3], b[(k >> 1) & 3], acc[k], 0, 0, 0);
    }
    int32_t x = 0;
#pragma unroll
    for (int k = 0; k < CEIL_ACC; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) x ^= acc[k][r];
    out[blockIdx.x * (64 * CEIL_WAVES) + threadIdx.x] = x;
    if (stamp && stamp_end) {
        clk[2] = (int64_t)__builtin_amdgcn_s_memtime();
        clk[3] = (int64_t)__builtin_amdgcn_s_memrealtime();
    }
}

// int8 MACs of one launch of `iters` trips (rounded up to a multiple of 4).
double ceiling_macs(int grid, int iters)
{
    const int trips = (iters + 3) / 4 * 4;
    return (double)grid * CEIL_WAVES * trips * CEIL_ACC * (32.0 * 32.0 * 32.0);
}

int ceiling_threads() { return 64 * CEIL_WAVES; }

hipError_t launch_mfma_ceiling(int grid, int iters, int32_t *out, int64_t *clk, bool stamp_start, bool stamp_end,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(mfma_ceiling, dim3(grid), dim3(64 * CEIL_WAVES), 0, stream, iters, out, clk,
                       stamp_start ? 1 : 0, stamp_end ? 1 : 0);
    return hipGetLastError();
}

}  // namespace xeng
