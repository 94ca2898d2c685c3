"""GPU parity of batched launches: many channels and sub-arrays of uneven N
and T in one persistent launch per kernel kind, prepared batches replayed
from a hipGraph (with their device-side integration guard), and the
autotuner.  Every result is compared bit for bit with the CPU oracle (small
cases: run in the test; full-size cases: every visibility against the
oracle's recorded digest) and with the same job launched alone."""
import numpy as np
import pytest

import oracle
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


def alone(X, x, n=None):
    c = X.Correlator(x.shape[1] if n is None else n, 1)
    c.correlate(0, gpu(x))
    v = c.dump(0)
    c.close()
    return v


def test_mixed_batch_matches_oracle_and_alone(X):
    # both kernel kinds in one call: N % 16 == 0 jobs take the DMA kernel,
    # the others the general one
    shapes = [(256, 700), (100, 333), (512, 64), (64, 4096), (256, 1), (300, 129)]
    print("mixed batch", shapes, flush=True)
    xs = [synth.uniform_bytes(n, t, seed=500 + i) for i, (n, t) in enumerate(shapes)]
    cs = [X.Correlator(n, 2) for n, _ in shapes]
    X.correlate_batch([(c, 1, gpu(x)) for c, x in zip(cs, xs)])
    for c, x in zip(cs, xs):
        v = c.dump(1)
        np.testing.assert_array_equal(v.cpu().numpy(), oracle.correlate(x))
        assert torch.equal(v, alone(X, x))
        assert not c.dump(0).any()      # the other slot is untouched
        c.close()


def test_batch_channels_reduced(X):
    # batched channels, at N = 256: uneven T, 5% of inputs flagged
    chans = synth.batched_channels(n_channels=16, n_inputs=256, t_lo=2048, t_hi=4096, seed=3)
    print("batched channels n=256", [x.shape[0] for x in chans], flush=True)
    c = X.Correlator(256, 16)
    X.correlate_batch([(c, k, gpu(x)) for k, x in enumerate(chans)])
    for k, x in enumerate(chans):
        np.testing.assert_array_equal(c.dump(k).cpu().numpy(), oracle.correlate(x))


def test_subarray_batch_reduced(X):
    subs = synth.subarray_batch(n_instances=24, n_choices=(256, 512, 100), t_choices=(64, 500, 1024),
                                seed=4)
    print("subarray batch", [x.shape for x in subs], flush=True)
    cs = [X.Correlator(x.shape[1], 1) for x in subs]
    X.correlate_batch([(c, 0, gpu(x)) for c, x in zip(cs, subs)])
    for c, x in zip(cs, subs):
        np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(x))
        c.close()


def test_batch_channels_full_size(X):
    # 16 channels x N = 2048, T uniform in [2048, 16384], 5% flagged: one
    # batched launch; every channel's complete output against the oracle's
    # recorded digest and against the channel launched alone; flagged
    # inputs give zero rows and columns
    import parity_util as pu
    chans = pu.fc.channels16()
    print("batched channels full size", [x.shape[0] for x in chans], flush=True)
    c = X.Correlator(2048, 16)
    X.correlate_batch([(c, k, gpu(x)) for k, x in enumerate(chans)])
    n = 2048
    for k, x in enumerate(chans):
        v = c.dump(k)
        pu.assert_matches_oracle_digest(f"channels16_c{k}", v, x)
        assert torch.equal(v, alone(X, x))
        flagged = np.where((x == 0x88).all(axis=0))[0]
        assert len(flagged) >= 102
        i = int(flagged[0])
        row = [oracle.tri_index(min(i, j), max(i, j), n) for j in range(n)]
        assert not v[row].any()


def test_subarray_batch_full_size(X):
    # 64 sub-arrays of uneven N and T in one batched launch: every
    # instance's complete output against the oracle's recorded digest and
    # against the instance launched alone
    import parity_util as pu
    subs = pu.fc.subarrays64()
    print("subarray batch full size", sum(x.nbytes for x in subs) / 1e6, "MB", flush=True)
    cs = [X.Correlator(x.shape[1], 1) for x in subs]
    X.correlate_batch([(c, 0, gpu(x)) for c, x in zip(cs, subs)])
    for k, (c, x) in enumerate(zip(cs, subs)):
        v = c.dump(0)
        pu.assert_matches_oracle_digest(f"subarrays64_k{k}", v, x)
        assert torch.equal(v, alone(X, x))
        c.close()


def test_batch_rejects_bad_jobs(X):
    c = X.Correlator(64, 2)
    x = gpu(synth.uniform_bytes(64, 10, seed=1))
    with pytest.raises(X.XengError) as e:
        X.correlate_batch([(c, 0, x), (c, 0, x)])          # same slot twice
    assert e.value.status == X.XENG_EINVAL
    big = torch.zeros((X.max_integration(), 64), dtype=torch.uint8, device="cuda")
    X.correlate_batch([(c, 1, big)])
    with pytest.raises(X.XengError) as e:
        X.correlate_batch([(c, 0, x), (c, 1, x)])          # slot 1 would overflow
    assert e.value.status == X.XENG_EOVERFLOW
    assert c.samples_integrated(0) == 0                     # nothing queued
    del big
    c.close()


def test_prepared_batch_graph_replays(X):
    # a prepared batch captured in a hipGraph: every replay integrates the
    # jobs again and advances the slots' device counters; each replay is
    # checked against the oracle, with eager work and synchronizations
    # between replays
    shapes = [(256, 300), (512, 129), (100, 77)]
    xs = [synth.uniform_bytes(n, t, seed=900 + i) for i, (n, t) in enumerate(shapes)]
    refs = [oracle.correlate(x) for x in xs]
    cs = [X.Correlator(n, 1) for n, _ in shapes]
    bufs = [gpu(x) for x in xs]
    b = X.Batch([(c, 0, t) for c, t in zip(cs, bufs)])
    b.launch()                                              # eager launch
    for c, r in zip(cs, refs):
        np.testing.assert_array_equal(c.dump(0, reset=False).cpu().numpy(), r)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.launch(stream=s)
    assert [c.samples_integrated(0) for c in cs] == [t for _, t in shapes]   # capture adds nothing
    other = X.Correlator(64, 1)
    y = gpu(synth.uniform_bytes(64, 100, seed=3))
    for rep in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        for c, r in zip(cs, refs):
            np.testing.assert_array_equal(c.dump(0, reset=False).cpu().numpy(), (rep + 1) * r)
        assert [c.samples_integrated(0) for c in cs] == [(rep + 1) * t for _, t in shapes]
        other.correlate(0, y)                               # eager work between replays
        torch.cuda.synchronize()
    assert b.check() == X.XENG_OK
    b.close()
    # the count is the host's again after the batch is gone
    assert [c.samples_integrated(0) for c in cs] == [4 * t for _, t in shapes]
    for c in cs:
        c.close()


def test_prepared_batch_guard_refuses_replay_past_bound(X):
    # a slot brought within one job of the integration bound: a replay that
    # fits integrates, the next (which would pass the bound) is refused on
    # the device -- accumulators and counter unchanged, reported by check()
    # -- and an eager call into the slot afterwards still adds to what the
    # replays integrated (the slot is never taken for an empty one)
    n, job = 64, 64
    tmax = X.max_integration()
    zeros = torch.zeros((1 << 20, n), dtype=torch.uint8, device="cuda")   # every sample -8-8j
    c = X.Correlator(n, 1)
    done, target = 0, tmax - job - 10
    while done < target:
        k = min(zeros.shape[0], target - done)
        c.correlate(0, zeros[:k])
        done += k
    x = gpu(np.zeros((job, n), dtype=np.uint8))
    b = X.Batch([(c, 0, x)])
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.launch(stream=s)
    g.replay()                                          # fits: tmax - 10
    torch.cuda.synchronize()
    assert c.samples_integrated(0) == tmax - 10
    assert b.check() == X.XENG_OK
    g.replay()                                          # would pass the bound
    torch.cuda.synchronize()
    assert b.check() == X.XENG_EOVERFLOW
    assert b.check() == X.XENG_OK                       # reported once
    assert c.samples_integrated(0) == tmax - 10
    v = c.dump(0, reset=False).cpu().numpy().astype(np.int64)
    assert (v[:, 0] == 128 * (tmax - 10)).all() and not v[:, 1].any()
    # eager call on the bound slot: guard from the device count, adds
    with pytest.raises(X.XengError) as e:
        c.correlate(0, zeros[:11])
    assert e.value.status == X.XENG_EOVERFLOW
    u = synth.uniform_bytes(n, 10, seed=91)
    c.correlate(0, gpu(u))
    assert c.samples_integrated(0) == tmax
    v = c.dump(0, reset=False).cpu().numpy().astype(np.int64)
    ref = oracle.correlate(u)
    np.testing.assert_array_equal(v[:, 0], 128 * (tmax - 10) + ref[:, 0])
    np.testing.assert_array_equal(v[:, 1], ref[:, 1])
    # after a reset the replays fit again
    c.reset(0)
    g.replay()
    torch.cuda.synchronize()
    assert b.check() == X.XENG_OK and c.samples_integrated(0) == job
    assert (c.dump(0, reset=False).cpu().numpy()[:, 0] == 128 * job).all()
    b.close()
    assert c.samples_integrated(0) == job
    c.close()


def test_autotune_keeps_results(X):
    # the slots hold integrated data before the autotuner runs: it times on
    # accumulators of its own and leaves them (and their counts) as they were
    shapes = [(512, 2000), (256, 3000), (128, 1000)]
    xs = [synth.uniform_bytes(n, 2 * t, seed=700 + i) for i, (n, t) in enumerate(shapes)]
    cs = [X.Correlator(n, 1) for n, _ in shapes]
    first = [(c, 0, gpu(x[:t])) for c, x, (_, t) in zip(cs, xs, shapes)]
    second = [(c, 0, gpu(x[t:])) for c, x, (_, t) in zip(cs, xs, shapes)]
    try:
        X.correlate_batch(first)
        torch.cuda.synchronize()
        before = [c.dump(0, reset=False).cpu().numpy() for c in cs]
        best = X.autotune(second, iters=2)
        print("autotuned", best, flush=True)
        assert best.kernel in (X.XENG_KERNEL_AUTO, X.XENG_KERNEL_GENERAL, X.XENG_KERNEL_DMA4)
        assert best.wgs_per_cu in (1, 2) and best.min_stages >= 1 and best.us_per_launch > 0
        assert best.source == X.XENG_TUNE_MEASURED and best.saved
        for c, b, (_, t) in zip(cs, before, shapes):
            assert c.samples_integrated(0) == t
            np.testing.assert_array_equal(c.dump(0, reset=False).cpu().numpy(), b)
        assert X.tuning_lookup(second).source == X.XENG_TUNE_MEASURED
        X.correlate_batch(second)                              # now with the tuned configuration
        for c, x in zip(cs, xs):
            np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(x))
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)                # defaults; drops the tuned entry
        for c in cs:
            c.close()


def test_batch_pads_jobs_the_dma_kernel_cannot_read(X):
    # N >= 256 that the DMA kernel cannot read in place (N not a multiple of
    # 16, or an odd stride or base) is copied into padded rows for the batched
    # launch; a DMA-ready job and a small general-kernel job ride along
    shapes = [(1000, 700), (2047, 129), (300, 64), (256, 100), (100, 50)]
    print("padded batch", shapes, flush=True)
    xs = [synth.uniform_bytes(n, t, seed=[700, n, t]) for n, t in shapes]
    # one more job: a misaligned view with an odd row stride
    big = synth.uniform_bytes(523, 257, seed=701)
    view = gpu(big)[:, 3:3 + 512]
    cs = [X.Correlator(n, 1) for n, _ in shapes] + [X.Correlator(512, 1)]
    X.correlate_batch([(c, 0, gpu(x)) for c, x in zip(cs, xs)] + [(cs[-1], 0, view)])
    for c, x in zip(cs, xs + [big[:, 3:3 + 512]]):
        v = c.dump(0)
        np.testing.assert_array_equal(v.cpu().numpy(), oracle.correlate(np.ascontiguousarray(x)))
        c.close()
