// Allocation-free correlation (xeng_correlate_static): the plan of a
// single-channel call -- the pieces each workgroup of the persistent launch
// runs, and their per-workgroup offsets -- is written by a one-thread
// device kernel into a fixed device array instead of memory the library
// allocates and caches.  The correlation kernels then read it exactly as
// they read a cached plan.
#include <hip/hip_runtime.h>

#include "xeng_internal.h"
#include "xeng_plan_single.h"

namespace xeng {

// Size of the array, bytes; xeng.h states the same limit.
constexpr int64_t STATIC_SCRATCH = INT64_C(1) << 20;

// One copy per GPU, held until the process ends.  Host code must use the
// device address returned by static_scratch_address(), never this name.
static __device__ __align__(256) uint8_t scratch[STATIC_SCRATCH];

// Device address of this GPU's scratch array.  Called once per device, with
// that device current, when the library sets the device up.
hipError_t static_scratch_address(void **ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

// The plan of one job: pieces in workgroup order (the order single_fill
// emits them), pieces of a unit cut into several flagged atomic, and the
// offsets wg_off[0 .. used].  One thread: the planner's greedy fill is
// sequential, and a plan has at most a few thousand pieces.
__global__ void static_plan(SinglePlanArgs a, Piece *__restrict__ pieces, int32_t *__restrict__ wg_off,
                            int32_t used)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int32_t w = 0; w <= used; ++w) wg_off[w] = 0;
    int64_t np = 0, unit_first = 0;
    auto close_unit = [&]() {
        if (np - unit_first > 1)
            for (int64_t q = unit_first; q < np; ++q) pieces[q].t1_atomic |= (int32_t)0x80000000u;
        unit_first = np;
    };
    single_fill(a, [&](int64_t w, int32_t ti, int32_t tj, int64_t s0, int64_t s1, int64_t k) {
        if (k == 0) close_unit();
        Piece p;
        p.job = 0;
        p.tile = ti | (tj << 16);
        p.t0 = (int32_t)(s0 * STAGE);
        p.t1_atomic = (int32_t)(s1 * STAGE < a.t ? s1 * STAGE : a.t);
        pieces[np++] = p;
        wg_off[w + 1] += 1;
    });
    close_unit();
    for (int32_t w = 0; w < used; ++w) wg_off[w + 1] += wg_off[w];
}

hipError_t launch_static_plan(const SinglePlanArgs &a, Piece *pieces, int32_t *wg_off, int32_t used,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(static_plan, dim3(1), dim3(64), 0, stream, a, pieces, wg_off, used);
    return hipGetLastError();
}

}  // namespace xeng
