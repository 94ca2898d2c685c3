"""Host-side checks of the C ABI library: it loads, exports every symbol the
header declares, validates arguments before touching the device, and its
work decomposition covers every (pair, sample) exactly once."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xeng.h")


@pytest.fixture(scope="module")
def X():
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xeng_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(X):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(X.lib(), name), name


def test_constants(X):
    assert X.max_integration() == (2 ** 31 - 1) // 128 == 16_777_215
    assert X.slot_bytes(0) == -1
    # tile-major accumulators: tri(ceil(N/128)) tiles of 128 x 128 x (Re, Im) int32
    for n in (1, 128, 129, 2048):
        nt = -(-n // 128)
        assert X.slot_bytes(n) == nt * (nt + 1) // 2 * 128 * 128 * 8 + 4 * (-(-n // 64) * 64)
    assert X.strerror(0) == "ok"
    assert "exact int32" in X.strerror(X.XENG_EOVERFLOW)


def test_argument_checks_without_device(X):
    L = X.lib()
    h = ctypes.c_void_p()
    assert L.xeng_create(None, ctypes.byref(h)) == X.XENG_EINVAL
    for bad in (X._Config(0, 1, 0, 0, 0), X._Config(8, 0, 0, 0, 0),
                X._Config(8, 1, -1, 0, 0), X._Config(8, 1, 0, 8, 0),
                X._Config(8, 1, 0, 0, -5)):
        assert L.xeng_create(ctypes.byref(bad), ctypes.byref(h)) == X.XENG_EINVAL
    # a memory budget below one slot is refused before any allocation
    cfg = X._Config(2048, 4, 0, 0, X.slot_bytes(2048) * 4 - 1)
    assert L.xeng_create(ctypes.byref(cfg), ctypes.byref(h)) == X.XENG_ENOMEM
    assert L.xeng_correlate(None, 0, None, 10, 10, None) == X.XENG_EINVAL
    assert L.xeng_dump(None, 0, None, 1, None) == X.XENG_EINVAL
    assert L.xeng_reset(None, 0, None) == X.XENG_EINVAL
    assert L.xeng_destroy(None) == X.XENG_EINVAL
    assert L.xeng_samples_integrated(None, 0) == -1
    assert L.xeng_correlate_batch(None, 1, None) == X.XENG_EINVAL
    assert L.xeng_correlate_batch(None, 0, None) == X.XENG_OK
    assert L.xeng_correlate_reference(None, 10, 4, 4, 0, None, None) == X.XENG_EINVAL
    assert L.xeng_set_tuning(3, 0, -1) == X.XENG_EINVAL
    assert L.xeng_set_tuning(0, 0, 7) == X.XENG_EINVAL
    assert L.xeng_clock_probe(-1, None) == X.XENG_EINVAL
    assert L.xeng_dump_batch(None, 1, None) == X.XENG_EINVAL
    assert L.xeng_dump_batch(None, 0, None) == X.XENG_OK
    no_ctx = (X._DumpJob * 1)()
    assert L.xeng_dump_batch(no_ctx, 1, None) == X.XENG_EINVAL
    # server configurations are checked before any device call: unknown flag
    # bits, a zero export cadence and a nonzero reserved field are refused
    for flags, dump, reserved in ((4, 8, 0), (1 << 31, 8, 0), (0, 0, 0), (X.XENG_SERVER_STAGGER_EXPORTS, 8, 1)):
        sc = X._ServerConfig(64, 0, flags, 256, dump, 16, 2, 4, 655.36, 1000.0, 0, reserved)
        assert L.xeng_server_create(ctypes.byref(sc), ctypes.byref(h)) == X.XENG_EINVAL


def _check_cover(pieces, jobs, grid):
    """Every (job, accumulator tile, sample) covered by exactly one piece."""
    cover = {}
    per_wg = {}
    n_pieces = {}
    for p in pieces:
        assert 0 <= p.workgroup < grid
        n, t = jobs[p.job]
        nt = -(-n // 128)
        assert p.n_tiles in (1, 2)
        assert p.ti <= p.tj + p.n_tiles - 1 and p.tj < nt
        assert 0 <= p.t0 < p.t1 <= t
        assert p.t0 % 64 == 0
        for tj in range(p.tj, p.tj + p.n_tiles):
            if p.ti <= tj < nt:          # stored tiles only
                cover.setdefault((p.job, p.ti, tj), []).append((p.t0, p.t1, p.atomic))
        per_wg[p.workgroup] = per_wg.get(p.workgroup, 0) + -(-(p.t1 - p.t0) // 64)
        n_pieces[p.workgroup] = n_pieces.get(p.workgroup, 0) + 1
    for j, (n, t) in enumerate(jobs):
        nt = -(-n // 128)
        for ti in range(nt):
            for tj in range(ti, nt):
                segs = sorted(cover.get((j, ti, tj), []))
                if t == 0:
                    assert not segs
                    continue
                assert segs, (j, ti, tj)
                assert segs[0][0] == 0 and segs[-1][1] == t
                for a, b in zip(segs, segs[1:]):
                    assert a[1] == b[0]
                assert all(s[2] == (len(segs) > 1) for s in segs)
    return per_wg, n_pieces


def stage_cost(p, n, wide):
    """The planners' cost of one stage of a piece's unit, in sixteenths: a
    wide window with one of its two tiles outside the triangle (below the
    diagonal, or past the last tile column) costs 13, any other unit 16."""
    if not wide:
        return 16
    nt = -(-n // 128)
    vl = p.ti <= p.tj < nt
    vr = p.ti <= p.tj + 1 < nt
    return 13 if vl != vr else 16


def test_half_windows_are_costed_lower(X):
    # N = 2048: the eight windows of the odd tile rows that start one tile
    # left of the diagonal are the only half windows; the linear plan gives
    # their workgroups more stages than the others
    X.set_plan_order(X.XENG_PLAN_LINEAR)
    try:
        pieces = X.plan_inspect([2048], [32768], 256, 4, True)
    finally:
        X.set_plan_order(X.XENG_PLAN_XCD)
    half = {(p.ti, p.tj) for p in pieces if stage_cost(p, 2048, True) == 13}
    assert half == {(ti, ti - 1) for ti in range(1, 16, 2)}
    st_half = [p.t1 - p.t0 for p in pieces if (p.ti, p.tj) in half]
    st_full = [p.t1 - p.t0 for p in pieces if (p.ti, p.tj) not in half]
    assert max(st_half) > max(st_full)


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("jobs,grid,min_st", [
    ([(2048, 32768)], 512, 8),
    ([(2048, 32768)], 256, 8),
    ([(64, 4096)], 512, 8),
    ([(1, 1)], 512, 8),
    ([(129, 33)], 7, 1),
    ([(300, 1000), (5, 0), (1024, 16384), (256, 4097)], 512, 4),
])
def test_plan_covers_exactly_once(X, jobs, grid, min_st, wide):
    X.set_plan_order(X.XENG_PLAN_LINEAR)
    try:
        pieces = X.plan_inspect([j[0] for j in jobs], [j[1] for j in jobs], grid, min_st, wide)
    finally:
        X.set_plan_order(X.XENG_PLAN_XCD)
    stages, n_pieces = _check_cover(pieces, jobs, grid)
    # balance: the cost of a workgroup -- its stages, each weighted by its
    # unit's stage cost, plus a fixed overhead per piece (prologue and
    # flush) -- is within one overhead and one stage of every other's; only
    # the last workgroup may have less
    ovh = (16 if wide else 8) * 16
    ws = sorted(stages)
    assert ws == list(range(len(ws)))
    cost = {w: ovh * n_pieces[w] for w in ws}
    for p in pieces:
        cost[p.workgroup] += (p.t1 - p.t0 + 63) // 64 * stage_cost(p, jobs[p.job][0], wide)
    cost = np.array([cost[w] for w in ws])
    if len(cost) > 2:
        assert cost[:-1].max() - cost[:-1].min() <= ovh + 16
        assert cost[-1] <= cost[:-1].max()


@pytest.mark.parametrize("jobs,grid,min_st", [
    ([(64, 4096)], 512, 1), ([(64, 4096)], 512, 4), ([(16, 1), (48, 65), (64, 100_000)], 512, 4),
    ([(64, 4096)] * 300, 512, 4), ([(32, 63)], 7, 1),
])
def test_narrow_plan_covers_exactly_once(X, jobs, grid, min_st):
    # narrow units (N <= 64): one 64 x 64 region per job, pieces of at most
    # 1023 stages, a grid of at most 16 workgroups per unit
    pieces = X.plan_inspect([j[0] for j in jobs], [j[1] for j in jobs], grid, min_st, 2)
    _check_cover(pieces, jobs, grid)
    assert all(p.ti == 0 and p.tj == 0 and p.n_tiles == 1 for p in pieces)
    assert max(p.t1 - p.t0 for p in pieces) <= 1023 * 64
    assert len({p.workgroup for p in pieces}) <= 16 * len(jobs)
    L = X.lib()
    ni = (ctypes.c_int32 * 1)(65)
    ns = (ctypes.c_int64 * 1)(100)
    assert L.xeng_plan_inspect(ni, ns, 1, 8, 1, 2, None, 0) == X.XENG_EINVAL   # N > 64 is not narrow


def test_plan_random_batches(X):
    rng = np.random.default_rng(0)
    for _ in range(20):
        k = int(rng.integers(1, 6))
        jobs = [(int(rng.integers(1, 700)), int(rng.integers(0, 5000))) for _ in range(k)]
        grid = int(rng.integers(1, 600))
        for wide in (False, True):
            pieces = X.plan_inspect([j[0] for j in jobs], [j[1] for j in jobs], grid,
                                    int(rng.integers(1, 10)), wide)
            _check_cover(pieces, jobs, grid)


@pytest.mark.parametrize("wide,cap", [(False, 16383), (True, 1023)])
def test_plan_caps_piece_length(X, wide, cap):
    # inside a piece the general kernel's B operands carry 16x the samples
    # (pieces below 2^20 samples), the DMA kernel's A and B both do (below 2^16)
    t = 3_000_000
    jobs = [(256, t)]
    pieces = X.plan_inspect([256], [t], 1, 1, wide)
    _check_cover(pieces, jobs, 1)
    limit = (1 << 16) - 1 if wide else (1 << 20) - 1
    assert max(p.t1 - p.t0 for p in pieces) <= limit
    per_unit = -(-t // (cap * 64))
    # units of N = 256: tiles (0,0), (0,1), (1,1); wide tiles (0,0), (1,0)
    assert len(pieces) == (2 if wide else 3) * per_unit
    assert all(p.atomic for p in pieces)


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("n,t,grid,min_st", [
    (2048, 32768, 256, 4), (2048, 32768, 512, 8), (64, 4096, 256, 4), (1, 1, 256, 4),
    (129, 33, 7, 1), (1000, 3000, 256, 4), (256, 3_000_000, 1, 1), (2048, 16_777_215, 256, 4),
])
def test_static_planner_equals_cached_plan(X, n, t, grid, min_st, wide):
    # the allocation-free path's planner (written without containers, run by
    # a one-thread kernel) emits the same pieces as the cached planner's
    # linear order for a single job, and they cover every (pair, sample)
    # exactly once
    X.set_plan_order(X.XENG_PLAN_LINEAR)
    try:
        want = X.plan_inspect([n], [t], grid, min_st, wide)
    finally:
        X.set_plan_order(X.XENG_PLAN_XCD)
    got = X.plan_inspect_static(n, t, grid, min_st, wide)
    assert got == want
    _check_cover(got, [(n, t)], grid)


def test_static_planner_rejects_bad_arguments(X):
    L = X.lib()
    assert L.xeng_plan_inspect_static(0, 10, 1, 1, 0, None, 0) == X.XENG_EINVAL
    assert L.xeng_plan_inspect_static(10, 0, 1, 1, 0, None, 0) == X.XENG_EINVAL
    assert L.xeng_plan_inspect_static(10, 10, 0, 1, 0, None, 0) == X.XENG_EINVAL
    assert L.xeng_plan_inspect_static(10, 10, 1, 1, 2, None, 0) == X.XENG_EINVAL
    assert L.xeng_plan_inspect_static(10, X.max_integration() + 1, 1, 1, 0, None, 0) == X.XENG_EINVAL
    assert L.xeng_correlate_static(None, 0, None, 10, 10, None) == X.XENG_EINVAL


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("n,t,grid", [(2048, 32768, 256), (2048, 32768, 512), (2000, 32768, 256),
                                      (1024, 32768, 256), (2048, 16384, 256), (1536, 65536, 256),
                                      (2048, 4096, 256), (256, 5000, 64), (2048, 16_777_215, 256)])
def test_xcd_plan_covers_exactly_once_and_balances(X, n, t, grid, wide):
    # the XCD-aware order (the default for single jobs): every (pair, sample)
    # exactly once, no workgroup costlier (in unweighted stages) than under
    # the linear order by more than one piece overhead, and where it applies
    # the main segments
    # of the 32 workgroups of one XCD (physical id % 8) share a time window
    pieces = X.plan_inspect([n], [t], grid, 4, wide)
    stages, n_pieces = _check_cover(pieces, [(n, t)], grid)
    ovh = 16 if wide else 8
    X.set_plan_order(X.XENG_PLAN_LINEAR)
    try:
        lin = X.plan_inspect([n], [t], grid, 4, wide)
    finally:
        X.set_plan_order(X.XENG_PLAN_XCD)
    lin_stages, lin_pieces = _check_cover(lin, [(n, t)], grid)
    cost = max(stages[w] + ovh * n_pieces[w] for w in stages)
    lin_cost = max(lin_stages[w] + ovh * lin_pieces[w] for w in lin_stages)
    assert cost <= lin_cost + ovh
    if (n, t, grid, wide) == (2048, 32768, 256, True):
        last = {}
        for p in pieces:
            last[p.workgroup] = p            # a workgroup's last piece is its main segment
        for x in (0, 1, 3, 5, 7):            # XCDs wholly inside one window (full units;
            # a half window's segments are longer, for the same cost)
            assert len({last[w].t0 for w in range(x, grid, 8) if stage_cost(last[w], n, wide) == 16}) == 1
