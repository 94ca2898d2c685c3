// Stream-K decomposition of ONE job, written without containers so that the
// same code runs on the host (sizing the plan, finding its budget) and in a
// one-thread device kernel that writes the plan straight into device
// memory.  It walks the job's units in the order plan_units gives and fills
// workgroups greedily exactly as make_plan does for a single job, so both
// produce the same pieces for the same budget.
#pragma once

#include "xeng_internal.h"

namespace xeng {

// Planner costs are in sixteenths of a stage of a full unit.  A wide unit
// (128 x 256 window of the DMA kernel) one of whose two tiles is not in the
// triangle -- the window of an odd tile row that starts one tile left of
// the diagonal, or one past the last tile column -- has four working
// regions instead of eight, which the kernel puts on four different SIMDs:
// half the matrix work per SIMD, but the same DMA, barriers and unpack
// latency per stage.  Costed at 13/16 of a full stage (measured best of
// 10/16 and 13/16 on N = 2048, T = 32768: 2.5 % fewer cycles per launch
// than costing them as full stages).
constexpr int64_t STAGE_COST = 16;
constexpr int64_t HALF_WINDOW_COST = 13;

__host__ __device__ inline int64_t unit_stage_cost(bool wide, int64_t ti, int64_t tj, int64_t nt)
{
    if (!wide) return STAGE_COST;
    const int64_t tjl = 2 * tj, tjr = tjl + 1;
    const bool vl = tjl >= ti && tjl < nt, vr = tjr >= ti && tjr < nt;
    return vl != vr ? HALF_WINDOW_COST : STAGE_COST;
}

struct SinglePlanArgs {
    int32_t n;          // inputs
    int64_t t;          // samples (> 0)
    int32_t wide;       // 1: 128 x 256 units (DMA kernel), 0: 128 x 128
    int64_t budget;     // per-workgroup cost: stage costs + overhead per piece
    int64_t overhead;   // cost charged per piece
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
            const int64_t wc = unit_stage_cost(a.wide != 0, ti, tj, nt);
            int64_t done = 0, k = 0;
            while (done < ns) {
                if (left - a.overhead < wc) {
                    if (++w >= a.grid) return a.grid + 1;
                    left = a.budget;
                }
                int64_t take = ns - done;
                if ((left - a.overhead) / wc < take) take = (left - a.overhead) / wc;
                if (a.cap < take) take = a.cap;
                emit(w, (int32_t)ti, (int32_t)tj, done, done + take, k++);
                done += take;
                left -= take * wc + a.overhead;
            }
        }
    }
    return w + 1;
}

}  // namespace xeng
