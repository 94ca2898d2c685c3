// Stream-K style decomposition of the upper-triangle tiles into pieces.
#include "xeng_plan.h"

#include <algorithm>

namespace xeng {

std::vector<std::pair<int, int>> plan_units(int n, TileShape shape)
{
    std::vector<std::pair<int, int>> u;
    const int nt = n_tiles_side(n);
    if (shape == TileShape::Square) {
        for (int ti = 0; ti < nt; ++ti)
            for (int tj = ti; tj < nt; ++tj) u.emplace_back(ti, tj);
    } else {
        const int nj2 = (nt + 1) / 2;
        for (int ti = 0; ti < nt; ++ti)
            for (int j2 = ti / 2; j2 < nj2; ++j2) u.emplace_back(ti, j2);
    }
    return u;
}

// Cost of a piece beyond its stages, in stage units: its prologue (the
// first stages' loads are not yet overlapped) and its flush of the tile's
// accumulators to memory.  Measured on the DMA kernel's 128 x 256 tiles at
// about 16 stage times; a 128 x 128 tile flushes half as much.
int64_t piece_overhead(TileShape shape) { return shape == TileShape::Wide ? 16 : 8; }

namespace {

struct UnitRef {
    int job, ti, tj;
    int64_t ns;   // stages
    int64_t t;    // samples
};

// Greedy fill: workgroups in order, each taking pieces of the linear (job,
// unit, stage) order until its cost (stages + overhead per piece) would
// exceed `budget`.  Returns the number of workgroups used (or grid + 1 if
// the work does not fit), emitting pieces when `out` is given.
template <typename Emit>
int64_t fill(const std::vector<UnitRef> &units, int64_t budget, int64_t overhead, int64_t cap, int64_t grid,
             Emit emit)
{
    int64_t w = 0, left = budget;
    for (size_t u = 0; u < units.size(); ++u) {
        int64_t done = 0;
        while (done < units[u].ns) {
            if (left <= overhead) {
                if (++w >= grid) return grid + 1;
                left = budget;
            }
            const int64_t take = std::min({units[u].ns - done, left - overhead, cap});
            emit(w, u, done, done + take);
            done += take;
            left -= take + overhead;
        }
    }
    return w + 1;
}

}  // namespace

Plan make_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages, TileShape shape)
{
    Plan plan;
    if (min_stages < 1) min_stages = 1;
    if (max_wgs < 1) max_wgs = 1;
    const int64_t cap = shape == TileShape::Wide ? MAX_PIECE_STAGES_WIDE : MAX_PIECE_STAGES;
    const int64_t ovh = piece_overhead(shape);

    std::vector<UnitRef> units;
    int64_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].t <= 0 || jobs[j].n <= 0) continue;
        const int64_t ns = (jobs[j].t + STAGE - 1) / STAGE;
        for (const auto &unit : plan_units(jobs[j].n, shape)) {
            units.push_back(UnitRef{j, unit.first, unit.second, ns, jobs[j].t});
            total += ns;
        }
    }
    if (total == 0) {
        plan.grid = 0;
        plan.wg_off.assign(1, 0);
        return plan;
    }
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(max_wgs, (total + min_stages - 1) / min_stages));

    // Smallest per-workgroup budget with which the greedy fill fits in
    // `grid` workgroups (the fill is monotone in the budget).
    auto none = [](int64_t, size_t, int64_t, int64_t) {};
    int64_t lo = ovh + 1, hi = ovh + total + 1;   // hi always fits: one piece per unit at most... per workgroup
    hi = std::max(hi, (total + grid - 1) / grid + ovh * ((int64_t)units.size() + 1) + 1);
    while (fill(units, hi, ovh, cap, grid, none) > grid) hi *= 2;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (fill(units, mid, ovh, cap, grid, none) <= grid)
            hi = mid;
        else
            lo = mid + 1;
    }

    struct Raw { Piece p; int32_t wg; size_t unit; };
    std::vector<Raw> raw;
    std::vector<int32_t> pieces_of_unit(units.size(), 0);
    const int64_t used = fill(units, lo, ovh, cap, grid, [&](int64_t w, size_t u, int64_t a, int64_t b) {
        Raw r;
        r.p.job = units[u].job;
        r.p.tile = units[u].ti | (units[u].tj << 16);
        r.p.t0 = (int32_t)(a * STAGE);
        r.p.t1_atomic = (int32_t)std::min<int64_t>(b * STAGE, units[u].t);
        r.wg = (int32_t)w;
        r.unit = u;
        raw.push_back(r);
        pieces_of_unit[u]++;
    });
    plan.grid = (int32_t)used;
    plan.wg_off.assign((size_t)used + 1, 0);
    // a tile cut into several pieces is flushed with atomics
    for (Raw &r : raw)
        if (pieces_of_unit[r.unit] > 1) r.p.t1_atomic |= (int32_t)0x80000000u;
    // pieces come out ordered by workgroup already
    plan.pieces.reserve(raw.size());
    plan.piece_wg.reserve(raw.size());
    for (const Raw &r : raw) {
        plan.pieces.push_back(r.p);
        plan.piece_wg.push_back(r.wg);
        plan.wg_off[(size_t)r.wg + 1]++;
    }
    for (size_t w = 0; w < (size_t)used; ++w) plan.wg_off[w + 1] += plan.wg_off[w];
    return plan;
}

SinglePlanArgs single_plan(int32_t n, int64_t t, TileShape shape, int max_wgs, int min_stages, int64_t *n_pieces,
                          int64_t *used)
{
    SinglePlanArgs a;
    a.n = n;
    a.t = t;
    a.wide = shape == TileShape::Wide ? 1 : 0;
    a.overhead = piece_overhead(shape);
    a.cap = shape == TileShape::Wide ? MAX_PIECE_STAGES_WIDE : MAX_PIECE_STAGES;
    if (min_stages < 1) min_stages = 1;
    if (max_wgs < 1) max_wgs = 1;
    const int64_t units = single_units(a);
    const int64_t total = units * single_stages(a);
    a.grid = std::max<int64_t>(1, std::min<int64_t>(max_wgs, (total + min_stages - 1) / min_stages));
    auto none = [](int64_t, int32_t, int32_t, int64_t, int64_t, int64_t) {};
    // the budget search of make_plan, over the same unit order
    int64_t lo = a.overhead + 1, hi = a.overhead + total + 1;
    hi = std::max(hi, (total + a.grid - 1) / a.grid + a.overhead * (units + 1) + 1);
    a.budget = hi;
    while (single_fill(a, none) > a.grid) a.budget = (hi *= 2);
    while (lo < hi) {
        a.budget = lo + (hi - lo) / 2;
        if (single_fill(a, none) <= a.grid)
            hi = a.budget;
        else
            lo = a.budget + 1;
    }
    a.budget = lo;
    int64_t np = 0;
    *used = single_fill(a, [&np](int64_t, int32_t, int32_t, int64_t, int64_t, int64_t) { ++np; });
    *n_pieces = np;
    return a;
}

}  // namespace xeng
