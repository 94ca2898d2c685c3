// Work decomposition of a (batched) correlation into per-workgroup pieces.
// Host only; no HIP dependency, so it is unit-testable without a GPU.
#pragma once

#include <stdint.h>
#include <utility>
#include <vector>

#include "xeng_internal.h"
#include "xeng_plan_single.h"

namespace xeng {

struct PlanJob {
    int32_t n;      // inputs
    int64_t t;      // samples
};

struct Plan {
    std::vector<Piece> pieces;      // grouped by workgroup
    std::vector<int32_t> wg_off;    // size grid + 1
    std::vector<int32_t> piece_wg;  // workgroup of each piece (for inspection)
    int32_t grid = 0;               // workgroups to launch
};

// Split the upper-triangle tiles of every job, each over its samples in
// STAGE-sample stages, into `max_wgs` (or fewer) nearly equal contiguous
// ranges of a linear (job, tile, stage) order: the stream-K decomposition.
// A tile cut into several pieces is marked atomic.  Every (i <= j, t) of
// every job is covered by exactly one piece.
//
// Square: units are the tiles (ti <= tj) of 128 x 128.  Wide: units are
// workgroup tiles (I, J2) of 128 rows x 256 columns, i.e. accumulator tiles
// (I, 2 J2) and (I, 2 J2 + 1), for every I <= 2 J2 + 1 (for I = 2 J2 + 1
// the left tile lies below the diagonal: the DMA kernel leaves it out).
// `cap` (stages), when positive, replaces the shape's longest piece.
Plan make_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages,
               TileShape shape = TileShape::Square, int64_t cap = 0);

// Units of one job in the plan's order: pairs (row index, column index)
// in the shape's own units.
std::vector<std::pair<int, int>> plan_units(int n, TileShape shape);

// XCD-aware, time-aligned decomposition of ONE job.  MI355X deals the
// workgroups of a launch to its 8 XCDs in turn (workgroup w on XCD w % 8),
// and each XCD has its own L2.  The job's units, in Morton order of their
// (row, column) tile coordinates, are cut into full time segments of L
// stages (L about the balanced share, total / grid) plus a tail each;
// logical workgroup k takes the k-th full segment in (time window, unit)
// order, and the tails are spread over the remaining workgroups by the
// stream-K fill.  Logical workgroups 32 x .. 32 x + 31 are placed on XCD x,
// so each XCD's workgroups work on one time window over a compact block of
// units and share those input rows and columns in its L2.  Every workgroup
// has one piece, or a few for the tails, as in the linear plan.  Returns
// false (nothing written) for a grid that is not a multiple of 8 or a job
// too short for one segment of XCD_MIN_SEGMENT stages per workgroup.
constexpr int XCDS = 8;
constexpr int64_t XCD_MIN_SEGMENT = 32;
bool make_plan_xcd(const PlanJob &job, int max_wgs, TileShape shape, Plan *out);

// Stage-equivalents charged per piece (prologue and flush) by the planners.
int64_t piece_overhead(TileShape shape);
// Longest piece of a shape's kernel, in stages: its int32 register sums
// stay exact (the general kernel's B operands carry 16x the samples, the
// DMA and narrow kernels' A and B operands both do).
int64_t piece_cap(TileShape shape);

// Plan parameters of one job as make_plan would choose them (grid and
// budget), for the container-free planner of xeng_plan_single.h; also the
// number of pieces and of workgroups used.  Host only, allocates nothing.
SinglePlanArgs single_plan(int32_t n, int64_t t, TileShape shape, int max_wgs, int min_stages, int64_t *n_pieces,
                          int64_t *used);

}  // namespace xeng
