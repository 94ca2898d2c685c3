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

Plan make_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages, TileShape shape)
{
    Plan plan;
    if (min_stages < 1) min_stages = 1;
    if (max_wgs < 1) max_wgs = 1;

    // Total work in stage units over all (job, tile) pairs.
    int64_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].t <= 0 || jobs[j].n <= 0) continue;
        const int64_t ns = (jobs[j].t + STAGE - 1) / STAGE;
        total += (int64_t)plan_units(jobs[j].n, shape).size() * ns;
    }
    if (total == 0) {
        plan.grid = 0;
        plan.wg_off.assign(1, 0);
        return plan;
    }
    const int64_t cap = shape == TileShape::Wide ? MAX_PIECE_STAGES_WIDE : MAX_PIECE_STAGES;
    int64_t grid = std::min<int64_t>(max_wgs, (total + min_stages - 1) / min_stages);
    grid = std::max<int64_t>(grid, 1);
    plan.grid = (int32_t)grid;
    plan.wg_off.assign((size_t)grid + 1, 0);

    // Workgroup w owns the linear stage range [bound(w), bound(w + 1)).
    auto bound = [&](int64_t w) { return (w * total) / grid; };

    struct Raw { Piece p; int32_t wg; };
    std::vector<Raw> raw;
    int64_t u = 0;   // linear stage offset of the current tile
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].t <= 0 || jobs[j].n <= 0) continue;
        const int64_t t = jobs[j].t;
        const int64_t ns = (t + STAGE - 1) / STAGE;
        for (const auto &unit : plan_units(jobs[j].n, shape)) {
            const int ti = unit.first, tj = unit.second;
            const int64_t lo = u, hi = u + ns;
            // first workgroup whose range intersects [lo, hi)
            int64_t w = (lo * grid) / total;
            while (w > 0 && bound(w) > lo) --w;
            while (bound(w + 1) <= lo) ++w;
            const size_t first = raw.size();
            for (; w < grid && bound(w) < hi; ++w) {
                const int64_t a = std::max(lo, bound(w)), b = std::min(hi, bound(w + 1));
                // long ranges are cut so that no piece exceeds the shape's cap
                for (int64_t c = a; c < b; c += cap) {
                    const int64_t e = std::min<int64_t>(b, c + cap);
                    Raw r;
                    r.p.job = j;
                    r.p.tile = ti | (tj << 16);
                    r.p.t0 = (int32_t)((c - lo) * STAGE);
                    r.p.t1_atomic = (int32_t)std::min<int64_t>((e - lo) * STAGE, t);
                    r.wg = (int32_t)w;
                    raw.push_back(r);
                }
            }
            if (raw.size() - first > 1)
                for (size_t k = first; k < raw.size(); ++k)
                    raw[k].p.t1_atomic |= (int32_t)0x80000000u;
            u = hi;
        }
    }
    // Raw pieces come out ordered by workgroup already (linear order).
    plan.pieces.reserve(raw.size());
    plan.piece_wg.reserve(raw.size());
    for (const Raw &r : raw) {
        plan.pieces.push_back(r.p);
        plan.piece_wg.push_back(r.wg);
        plan.wg_off[(size_t)r.wg + 1]++;
    }
    for (size_t w = 0; w < (size_t)grid; ++w) plan.wg_off[w + 1] += plan.wg_off[w];
    return plan;
}

}  // namespace xeng
