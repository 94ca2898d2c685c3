// Stream-K style decomposition of the upper-triangle tiles into pieces.
#include "xeng_plan.h"
#include "xeng_plan_single.h"

#include <algorithm>
#include <cstdint>
#include <unordered_map>

namespace xeng {

std::vector<std::pair<int, int>> plan_units(int n, TileShape shape)
{
    std::vector<std::pair<int, int>> u;
    const int nt = n_tiles_side(n);
    if (shape == TileShape::Narrow) {
        u.emplace_back(0, 0);
    } else if (shape == TileShape::Square) {
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

int64_t piece_cap(TileShape shape) { return shape == TileShape::Square ? MAX_PIECE_STAGES : MAX_PIECE_STAGES_WIDE; }

namespace {

struct UnitRef {
    int job, ti, tj;
    int64_t ns;   // stages
    int64_t t;    // samples
    int64_t wc;   // cost of one stage (unit_stage_cost)
};

// Greedy fill: workgroups in order, each taking pieces of the linear (job,
// unit, stage) order until its cost (stage costs + overhead per piece)
// would exceed `budget`.  Returns the number of workgroups used (or grid + 1 if
// the work does not fit), emitting pieces when `out` is given.
template <typename Emit>
int64_t fill(const std::vector<UnitRef> &units, int64_t budget, int64_t overhead, int64_t cap, int64_t grid,
             Emit emit)
{
    int64_t w = 0, left = budget;
    for (size_t u = 0; u < units.size(); ++u) {
        int64_t done = 0;
        const int64_t wc = units[u].wc;
        while (done < units[u].ns) {
            if (left - overhead < wc) {
                if (++w >= grid) return grid + 1;
                left = budget;
            }
            const int64_t take = std::min({units[u].ns - done, (left - overhead) / wc, cap});
            emit(w, u, done, done + take);
            done += take;
            left -= take * wc + overhead;
        }
    }
    return w + 1;
}

}  // namespace

Plan make_plan(const PlanJob *jobs, int n_jobs, int max_wgs, int min_stages, TileShape shape, int64_t cap_override)
{
    Plan plan;
    if (min_stages < 1) min_stages = 1;
    if (max_wgs < 1) max_wgs = 1;
    const int64_t cap = cap_override > 0 ? cap_override : piece_cap(shape);
    const int64_t ovh = piece_overhead(shape) * STAGE_COST;

    std::vector<UnitRef> units;
    int64_t total = 0, total_cost = 0;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].t <= 0 || jobs[j].n <= 0) continue;
        const int64_t ns = (jobs[j].t + STAGE - 1) / STAGE;
        const int64_t nt = n_tiles_side(jobs[j].n);
        for (const auto &unit : plan_units(jobs[j].n, shape)) {
            const int64_t wc = unit_stage_cost(shape == TileShape::Wide, unit.first, unit.second, nt);
            units.push_back(UnitRef{j, unit.first, unit.second, ns, jobs[j].t, wc});
            total += ns;
            total_cost += ns * wc;
        }
    }
    if (total == 0) {
        plan.grid = 0;
        plan.wg_off.assign(1, 0);
        return plan;
    }
    const int64_t grid = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)max_wgs, (total + min_stages - 1) / min_stages,
                              (int64_t)units.size() * MAX_UNIT_SPLIT}));

    // Smallest per-workgroup budget with which the greedy fill fits in
    // `grid` workgroups (the fill is monotone in the budget).
    auto none = [](int64_t, size_t, int64_t, int64_t) {};
    int64_t lo = ovh + STAGE_COST, hi = ovh + total_cost + 1;
    hi = std::max(hi, (total_cost + grid - 1) / grid + ovh * ((int64_t)units.size() + 1) + 1);
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

namespace {

// Interleaved bits of (a, b): units close in both coordinates come close
// together in this order, so a run of consecutive units covers a compact
// block of the triangle (few distinct row and column blocks).
uint64_t morton(uint32_t a, uint32_t b)
{
    uint64_t r = 0;
    for (int k = 0; k < 16; ++k) r |= (uint64_t)((a >> k) & 1u) << (2 * k + 1) | (uint64_t)((b >> k) & 1u) << (2 * k);
    return r;
}

}  // namespace

namespace {

// One candidate of make_plan_xcd for segment length L (in stages of a full
// unit): the pieces of each logical workgroup, and the largest workgroup
// cost (stage costs + overhead per piece, in sixteenths of a stage).  A
// unit whose stages cost less (`wc`) takes longer segments of the same
// cost.  Returns -1 if the work does not fit in G workgroups.
struct XSeg {
    int64_t u, s0, s1;
};

int64_t xcd_candidate(const std::vector<int64_t> &wc, int64_t ns, int64_t G, int64_t L, int64_t ovh, int64_t cap,
                      std::vector<std::vector<XSeg>> *out)
{
    const int64_t U = (int64_t)wc.size();
    std::vector<int64_t> Lu((size_t)U), Fu((size_t)U), ru((size_t)U);
    int64_t main = 0, max_f = 0, worst = 0;
    bool tails = false;
    for (int64_t u = 0; u < U; ++u) {
        Lu[(size_t)u] = std::min({ns, cap, std::max<int64_t>(1, L * STAGE_COST / wc[(size_t)u])});
        Fu[(size_t)u] = ns / Lu[(size_t)u];                  // full segments of the unit
        ru[(size_t)u] = ns - Fu[(size_t)u] * Lu[(size_t)u];  // its tail
        main += Fu[(size_t)u];
        max_f = std::max(max_f, Fu[(size_t)u]);
        tails = tails || ru[(size_t)u] > 0;
        if (Fu[(size_t)u] > 0) worst = std::max(worst, Lu[(size_t)u] * wc[(size_t)u] + ovh);
    }
    if (main > G || (tails && main == G)) return -1;
    if (out) {
        out->assign((size_t)G, {});
        int64_t k = 0;
        for (int64_t p = 0; p < max_f; ++p)
            for (int64_t u = 0; u < U; ++u)
                if (p < Fu[(size_t)u])
                    (*out)[(size_t)k++].push_back(XSeg{u, p * Lu[(size_t)u], (p + 1) * Lu[(size_t)u]});
    }
    if (!tails) return worst;
    // the tails: stream-K over the remaining workgroups, smallest budget that fits
    auto fill = [&](int64_t budget, bool emit) -> bool {
        int64_t k = main, left = budget, u = 0, done = 0;
        while (u < U) {
            const int64_t r = ru[(size_t)u], w = wc[(size_t)u];
            if (r == 0) {
                ++u;
                continue;
            }
            if (left - ovh < w) {
                if (++k >= G) return false;
                left = budget;
            }
            const int64_t take = std::min({r - done, (left - ovh) / w, cap});
            const int64_t base = Fu[(size_t)u] * Lu[(size_t)u];
            if (emit) (*out)[(size_t)k].push_back(XSeg{u, base + done, base + done + take});
            done += take;
            left -= take * w + ovh;
            if (done == r) {
                ++u;
                done = 0;
            }
        }
        return true;
    };
    int64_t lo = ovh + STAGE_COST, hi = ovh + STAGE_COST;
    while (!fill(hi, false)) hi *= 2;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (fill(mid, false))
            hi = mid;
        else
            lo = mid + 1;
    }
    if (out) fill(lo, true);
    return std::max(worst, lo);
}

}  // namespace

bool make_plan_xcd(const PlanJob &job, int max_wgs, TileShape shape, Plan *out)
{
    const int64_t G = max_wgs;
    if (G < XCDS || G % XCDS != 0 || job.n <= 0 || job.t <= 0 || shape == TileShape::Narrow) return false;
    std::vector<std::pair<int, int>> units = plan_units(job.n, shape);
    const int64_t U = (int64_t)units.size();
    const int64_t ns = (job.t + STAGE - 1) / STAGE;
    const int64_t ovh_st = piece_overhead(shape);
    const int64_t cap = shape == TileShape::Wide ? MAX_PIECE_STAGES_WIDE : MAX_PIECE_STAGES;
    const int col_scale = shape == TileShape::Wide ? 2 : 1;
    std::stable_sort(units.begin(), units.end(), [col_scale](const std::pair<int, int> &a, const std::pair<int, int> &b) {
        return morton((uint32_t)a.first, (uint32_t)(col_scale * a.second)) <
               morton((uint32_t)b.first, (uint32_t)(col_scale * b.second));
    });
    const int64_t nt = n_tiles_side(job.n);
    std::vector<int64_t> wc((size_t)U);
    int64_t total_cost = 0;
    for (int64_t u = 0; u < U; ++u) {
        wc[(size_t)u] = unit_stage_cost(shape == TileShape::Wide, units[(size_t)u].first, units[(size_t)u].second, nt);
        total_cost += ns * wc[(size_t)u];
    }
    // segment lengths around the balanced share (longer ones leave less
    // for the tail workgroups): the candidate with the smallest largest
    // workgroup cost wins
    const int64_t L0 = (total_cost + STAGE_COST * G - 1) / (STAGE_COST * G);
    if (L0 < XCD_MIN_SEGMENT || L0 >= ns) return false;
    int64_t best_L = -1, best_cost = -1;
    for (int64_t L = std::min({L0 + 4 * ovh_st, cap, ns - 1}); L >= std::max<int64_t>(XCD_MIN_SEGMENT, L0 - ovh_st);
         --L) {
        const int64_t c = xcd_candidate(wc, ns, G, L, ovh_st * STAGE_COST, cap, nullptr);
        if (c >= 0 && (best_cost < 0 || c < best_cost)) {
            best_cost = c;
            best_L = L;
        }
    }
    if (best_L < 0) return false;
    std::vector<std::vector<XSeg>> logical;
    xcd_candidate(wc, ns, G, best_L, ovh_st * STAGE_COST, cap, &logical);
    // a unit cut into several pieces is shared: flushed with atomics
    std::vector<int> pieces_of(units.size(), 0);
    for (const auto &v : logical)
        for (const XSeg &sg : v) pieces_of[(size_t)sg.u]++;
    // logical workgroup k runs on XCD k / (G / XCDS): physical id
    // (k % (G / XCDS)) * XCDS + k / (G / XCDS), workgroups being dealt to the
    // XCDs in turn
    const int64_t per_xcd = G / XCDS;
    std::vector<const std::vector<XSeg> *> by_wg((size_t)G);
    for (int64_t k = 0; k < G; ++k) by_wg[(size_t)((k % per_xcd) * XCDS + k / per_xcd)] = &logical[(size_t)k];
    Plan plan;
    plan.wg_off.assign((size_t)G + 1, 0);
    for (int64_t w = 0; w < G; ++w) {
        for (const XSeg &sg : *by_wg[(size_t)w]) {
            Piece pc;
            pc.job = 0;
            pc.tile = units[(size_t)sg.u].first | (units[(size_t)sg.u].second << 16);
            pc.t0 = (int32_t)(sg.s0 * STAGE);
            pc.t1_atomic = (int32_t)std::min<int64_t>(sg.s1 * STAGE, job.t);
            if (pieces_of[(size_t)sg.u] > 1) pc.t1_atomic |= (int32_t)0x80000000u;
            plan.pieces.push_back(pc);
            plan.piece_wg.push_back((int32_t)w);
        }
        plan.wg_off[(size_t)w + 1] = (int32_t)plan.pieces.size();
    }
    // every physical id up to G - 1 is launched (workgroups without pieces
    // return at once), so that the XCD placement holds
    plan.grid = (int32_t)G;
    *out = std::move(plan);
    return true;
}

SinglePlanArgs single_plan(int32_t n, int64_t t, TileShape shape, int max_wgs, int min_stages, int64_t *n_pieces,
                          int64_t *used)
{
    SinglePlanArgs a;
    a.n = n;
    a.t = t;
    a.wide = shape == TileShape::Wide ? 1 : 0;
    a.overhead = piece_overhead(shape) * STAGE_COST;
    a.cap = shape == TileShape::Wide ? MAX_PIECE_STAGES_WIDE : MAX_PIECE_STAGES;
    if (min_stages < 1) min_stages = 1;
    if (max_wgs < 1) max_wgs = 1;
    const int64_t units = single_units(a);
    const int64_t total = units * single_stages(a);
    a.grid = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)max_wgs, (total + min_stages - 1) / min_stages, units * MAX_UNIT_SPLIT}));
    auto none = [](int64_t, int32_t, int32_t, int64_t, int64_t, int64_t) {};
    // the budget search of make_plan, over the same unit order (total
    // stages at full cost bound the total cost from above)
    int64_t lo = a.overhead + STAGE_COST, hi = a.overhead + total * STAGE_COST + 1;
    hi = std::max(hi, (total * STAGE_COST + a.grid - 1) / a.grid + a.overhead * (units + 1) + 1);
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
