// Stream-K decomposition of ONE job, written without containers so that the
// same code runs on the host (sizing the plan, finding its budget) and in a
// one-thread device kernel that writes the plan straight into device
// memory.  It walks the job's units in the order plan_units gives and fills
// workgroups greedily exactly as make_plan does for a single job, so both
// produce the same pieces for the same budget.
#pragma once

#include "xeng_internal.h"

namespace xeng {

struct SinglePlanArgs {
    int32_t n;          // inputs
    int64_t t;          // samples (> 0)
    int32_t wide;       // 1: 128 x 256 units (DMA kernel), 0: 128 x 128
    int64_t budget;     // per-workgroup cost: stages + overhead per piece
    int64_t overhead;   // stage-equivalents charged per piece
    int64_t cap;        // longest piece, in stages
    int64_t grid;       // workgroups available
};

__host__ __device__ inline int64_t single_stages(const SinglePlanArgs &a) { return (a.t + STAGE - 1) / STAGE; }

__host__ __device__ inline int64_t single_units(const SinglePlanArgs &a)
{
    const int64_t nt = n_tiles_side_hd(a.n);
    if (!a.wide) return nt * (nt + 1) / 2;
    const int64_t nj2 = (nt + 1) / 2;
    int64_t u = 0;
    for (int64_t ti = 0; ti < nt; ++ti) u += nj2 - ti / 2;
    return u;
}

// Greedy fill: emit(w, ti, tj, first_stage, end_stage, unit_piece_index)
// for every piece in order; returns the workgroups used, or grid + 1 if the
// work does not fit in `grid` workgroups of `budget`.
template <typename Emit>
__host__ __device__ int64_t single_fill(const SinglePlanArgs &a, Emit &&emit)
{
    const int64_t nt = n_tiles_side_hd(a.n);
    const int64_t ns = single_stages(a);
    const int64_t nj2 = (nt + 1) / 2;
    int64_t w = 0, left = a.budget;
    for (int64_t ti = 0; ti < nt; ++ti) {
        const int64_t c0 = a.wide ? ti / 2 : ti, c1 = a.wide ? nj2 : nt;
        for (int64_t tj = c0; tj < c1; ++tj) {
            int64_t done = 0, k = 0;
            while (done < ns) {
                if (left <= a.overhead) {
                    if (++w >= a.grid) return a.grid + 1;
                    left = a.budget;
                }
                int64_t take = ns - done;
                if (left - a.overhead < take) take = left - a.overhead;
                if (a.cap < take) take = a.cap;
                emit(w, (int32_t)ti, (int32_t)tj, done, done + take, k++);
                done += take;
                left -= take + a.overhead;
            }
        }
    }
    return w + 1;
}

}  // namespace xeng
