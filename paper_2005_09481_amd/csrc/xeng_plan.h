// Work decomposition of a (batched) correlation into per-workgroup pieces.
// Host only; no HIP dependency, so it is unit-testable without a GPU.
#pragma once

#include <stdint.h>
#include <vector>

#include "xeng_internal.h"

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
Plan make_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages);

}  // namespace xeng
