"""GPU parity of the flag-aware path: spectral-kurtosis RFI flags, and the
flag-aware correlation's visibilities and per-pair sample counts, bit for
bit against the oracle (oracle/flags.py) -- small and ragged shapes, the
chunked copy, accumulation with unflagged calls, resets, and the full-size
N=2048, T=32768 channel with injected interference."""
import ctypes

import numpy as np
import pytest

import oracle
import oracle.flags as OF
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n,t,bl", [(1, 10, 2), (5, 100, 7), (64, 4096, 256), (100, 999, 64), (130, 3000, 1024),
                                    (2048, 1000, 256), (37, 513, 2)])
def test_rfi_flags_match_oracle(X, n, t, bl):
    print(f"rfi flags n={n} t={t} block={bl}", flush=True)
    x = synth.rfi_channel(n, t, seed=[21, n], block_len=bl, tone_frac=0.05, burst_frac=0.05)
    got = X.rfi_flags(gpu(x), block_len=bl).cpu().numpy()
    np.testing.assert_array_equal(got, OF.sk_flags(x, block_len=bl))


def test_rfi_flags_worked_example_thresholds_and_re_low(X):
    import test_oracle_flag_pins as P
    g = P._golden()
    x = np.array([[int(h, 16) for h in r.split()] for r in g["samples"]], dtype=np.uint8)
    f1 = X.rfi_flags(gpu(x), block_len=4, lo_num=625, hi_num=1375, den=1000).cpu().numpy()
    np.testing.assert_array_equal(f1[0], [int(v) for v in g["flags_625_1375"][0].split()])
    f2 = X.rfi_flags(gpu(x), block_len=4, lo_num=600, hi_num=4000, den=1000).cpu().numpy()
    np.testing.assert_array_equal(f2[0], [int(v) for v in g["flags_600_4000"][0].split()])
    # swapped nibbles with XENG_NIBBLE_RE_LOW: the same power, the same flags
    swapped = ((x & 15) << 4) | (x >> 4)
    f3 = X.rfi_flags(gpu(swapped), block_len=4, re_low=True).cpu().numpy()
    np.testing.assert_array_equal(f3, f1)
    # an odd stride and base (byte loads)
    y = synth.rfi_channel(70, 600, seed=22, block_len=50)
    big = np.zeros((600, 75), dtype=np.uint8)
    big[:, 3:73] = y
    view = gpu(big)[:, 3:73]
    np.testing.assert_array_equal(X.rfi_flags(view, block_len=50).cpu().numpy(), OF.sk_flags(y, block_len=50))


def run_flagged(X, x, fl, bl, n=None):
    n = x.shape[1] if n is None else n
    c = X.Correlator(n, 1, counts=True)
    c.correlate_flagged(0, gpu(x), gpu(fl), bl)
    cnt = c.dump_counts(0).cpu().numpy().astype(np.int64)
    vis = c.dump(0).cpu().numpy().astype(np.int64)
    assert not c.dump_counts(0).any()                    # the reset cleared the counts too
    c.close()
    return vis, cnt


@pytest.mark.parametrize("n,t,bl", [(1, 1, 1), (3, 10, 1), (16, 100, 3), (64, 4096, 256), (100, 1000, 64),
                                    (256, 333, 1), (300, 2000, 100), (1000, 3000, 256), (2047, 129, 40)])
def test_flagged_correlation_matches_oracle(X, n, t, bl):
    print(f"flagged correlation n={n} t={t} block={bl}", flush=True)
    rng = np.random.default_rng([23, n, t])
    x = synth.uniform_bytes(n, t, seed=[24, n, t])
    fl = (rng.random((OF.n_blocks(t, bl), n)) < 0.3).astype(np.uint8)
    vis, cnt = run_flagged(X, x, fl, bl)
    want_vis, want_cnt = OF.correlate_flagged(x, fl, bl)
    np.testing.assert_array_equal(vis, want_vis)
    np.testing.assert_array_equal(cnt, want_cnt)


def test_flagged_extremes_and_unflagged_equivalence(X):
    n, t, bl = 200, 1000, 64
    x = synth.uniform_bytes(n, t, seed=25)
    nb = OF.n_blocks(t, bl)
    vis, cnt = run_flagged(X, x, np.zeros((nb, n), np.uint8), bl)
    np.testing.assert_array_equal(vis, oracle.correlate(x))
    assert (cnt == t).all()
    vis, cnt = run_flagged(X, x, np.ones((nb, n), np.uint8), bl)
    assert not vis.any() and not cnt.any()


def test_flagged_accumulates_with_unflagged_calls_and_chunks(X):
    # flagged and plain calls into one slot: counts = flagged counts + the
    # plain calls' samples for every pair; the flagged call in several
    # chunks of the padded copy (the block index runs on across chunks)
    n, bl = 300, 50
    xs = [synth.uniform_bytes(n, t, seed=[26, t]) for t in (1000, 333, 777)]
    rng = np.random.default_rng(27)
    fls = [(rng.random((OF.n_blocks(x.shape[0], bl), n)) < 0.25).astype(np.uint8) for x in xs]
    try:
        X.set_pad_chunk_bytes(4 * 64 * 304)              # chunks of 256 rows
        c = X.Correlator(n, 2, counts=True)
        c.correlate_flagged(1, gpu(xs[0]), gpu(fls[0]), bl)
        c.correlate(1, gpu(xs[1]))
        c.correlate_flagged(1, gpu(xs[2]), gpu(fls[2]), bl)
        assert c.samples_integrated(1) == 1000 + 333 + 777
        v0, n0 = OF.correlate_flagged(xs[0], fls[0], bl)
        v2, n2 = OF.correlate_flagged(xs[2], fls[2], bl)
        np.testing.assert_array_equal(c.dump_counts(1).cpu().numpy(), n0 + 333 + n2)
        np.testing.assert_array_equal(c.dump(1, reset=False).cpu().numpy(), v0 + oracle.correlate(xs[1]) + v2)
        assert not c.dump_counts(0).any() and not c.dump(0).any()
        c.reset(1)
        assert not c.dump_counts(1).any()
        c.correlate(1, gpu(xs[1]))                       # plain calls alone: every pair counts T
        assert (c.dump_counts(1).cpu().numpy() == 333).all()
        c.close()
    finally:
        X.set_pad_chunk_bytes(0)


def test_flagged_argument_errors(X):
    L = X.lib()
    c = X.Correlator(64, 1)                              # no XENG_COUNTS
    x = gpu(synth.uniform_bytes(64, 10, seed=1))
    f = torch.zeros((1, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(X.XengError) as e:
        c.correlate_flagged(0, x, f, 16)
    assert e.value.status == X.XENG_EINVAL
    with pytest.raises(X.XengError):
        c.dump_counts(0)
    d = X.Correlator(64, 1, counts=True)
    assert L.xeng_correlate_flagged(d.handle, 0, ctypes.c_void_p(x.data_ptr()), 10, 64,
                                    ctypes.c_void_p(f.data_ptr()), 0, None) == X.XENG_EINVAL
    assert L.xeng_correlate_flagged(d.handle, 0, ctypes.c_void_p(x.data_ptr()), 10, 64, None, 16,
                                    None) == X.XENG_EINVAL
    cfg = X._RfiConfig(1, 1000, 625, 1375, 0)            # blocks of one sample: no estimator
    out = torch.zeros((10, 64), dtype=torch.uint8, device="cuda")
    assert L.xeng_rfi_flags(ctypes.c_void_p(x.data_ptr()), 10, 64, 64, 0, ctypes.byref(cfg),
                            ctypes.c_void_p(out.data_ptr()), None) == X.XENG_EINVAL
    cfg = X._RfiConfig(4, 1000, 1375, 625, 0)            # lo above hi
    assert L.xeng_rfi_flags(ctypes.c_void_p(x.data_ptr()), 10, 64, 64, 0, ctypes.byref(cfg),
                            ctypes.c_void_p(out.data_ptr()), None) == X.XENG_EINVAL
    assert d.samples_integrated(0) == 0
    c.close()
    d.close()


def test_full_size_flagged_channel(X):
    """N=2048, T=32768 with injected carriers and bursts, blocks of 256: the
    flags, every visibility and every pair count against the oracle."""
    n, t, bl = 2048, 32768, 256
    print("full-size flagged: generating", flush=True)
    x = synth.rfi_channel(n, t, seed=6, block_len=bl)
    xd = gpu(x)
    fl = X.rfi_flags(xd, block_len=bl)
    want_fl = OF.sk_flags(x, block_len=bl)
    np.testing.assert_array_equal(fl.cpu().numpy(), want_fl)
    print(f"full-size flagged: {want_fl.mean():.4f} of cells flagged", flush=True)
    c = X.Correlator(n, 1, counts=True)
    c.correlate_flagged(0, xd, fl, bl)
    cnt = c.dump_counts(0).cpu().numpy().astype(np.int64)
    vis = c.dump(0).cpu().numpy().astype(np.int64)
    c.close()
    want_vis, want_cnt = OF.correlate_flagged(x, want_fl, bl)
    np.testing.assert_array_equal(cnt, want_cnt)
    np.testing.assert_array_equal(vis, want_vis)
