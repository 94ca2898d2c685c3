"""GPU parity of the narrow kernel (N <= 64, a multiple of 16, 16-byte-aligned
rows): the four waves of a workgroup split the time of a piece and add
their partial sums through LDS before one flush.  Every visibility is
compared bit for bit with the CPU oracle: ragged T around the 64-sample
stage and the four-wave interleave, every N it serves, both nibble orders,
fresh and accumulating slots, pieces split across workgroups (atomic
flushes) and at the longest piece, extreme samples, strided rows, and
batches of many channels alone and mixed with wide and general jobs."""
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


def dump(c, slot=0):
    return c.dump(slot).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("n", [16, 32, 48, 64])
@pytest.mark.parametrize("t", [1, 63, 64, 65, 255, 256, 257, 1000, 4096, 5000])
def test_narrow_matches_oracle(X, n, t):
    print(f"narrow n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=4000 + n + t)
    c = X.Correlator(n, 1)
    try:
        c.correlate(0, gpu(x))
        np.testing.assert_array_equal(dump(c), oracle.correlate(x))
    finally:
        c.close()


@pytest.mark.parametrize("n", [16, 64])
def test_narrow_re_low_and_accumulation(X, n):
    # two calls on one slot: the first stores into the zeroed slot, the
    # second adds (read-modify-write); the low nibble as the real part
    x = synth.uniform_bytes(n, 3000, seed=4100 + n)
    c = X.Correlator(n, 1, re_low=True)
    try:
        c.correlate(0, gpu(x[:1300]))
        c.correlate(0, gpu(x[1300:]))
        np.testing.assert_array_equal(dump(c), oracle.correlate(x, re_low=True))
    finally:
        c.close()


@pytest.mark.parametrize("ms", [1, 4, 64, 1 << 20])
def test_narrow_pieces_split_and_longest(X, ms):
    # T = 100000 (1563 stages): beyond the longest piece (1023 stages), so
    # at least two pieces with atomic flushes; minimum piece lengths from 1
    # stage (16 workgroups per tile) to whole pieces.  Extreme samples make
    # the largest sums.
    n, t = 64, 100_000
    print(f"narrow split n={n} t={t} min_stages={ms}", flush=True)
    rng = np.random.default_rng(17)
    x = rng.choice(np.array([0x00, 0x0F, 0xF0, 0xFF, 0x80, 0x08], dtype=np.uint8), size=(t, n))
    c = X.Correlator(n, 1)
    try:
        X.set_tuning(0, ms, X.XENG_KERNEL_AUTO)
        c.correlate(0, gpu(x))
        np.testing.assert_array_equal(dump(c), oracle.correlate(x))
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
        c.close()


def test_narrow_extreme_at_the_longest_piece(X):
    # every sample (-8, -8): each pair sums 128 per sample; 65472 samples in
    # one piece (1023 stages) keep the register sums at 256 * 128 * 65472 <
    # 2^31
    n, t = 64, 1023 * 64
    x = np.full((t, n), 0x00, dtype=np.uint8)
    c = X.Correlator(n, 1)
    try:
        X.set_tuning(0, 1 << 20, X.XENG_KERNEL_AUTO)
        c.correlate(0, gpu(x))
        got = dump(c)
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
        c.close()
    np.testing.assert_array_equal(got, oracle.correlate(x))
    assert (got[:, 0] == 128 * t).all()


@pytest.mark.parametrize("n,stride", [(48, 64), (32, 48), (64, 80)])
def test_narrow_strided_rows(X, n, stride):
    t = 777
    full = synth.uniform_bytes(stride, t, seed=4200 + n)
    c = X.Correlator(n, 1)
    try:
        c.correlate(0, gpu(full)[:, :n])       # a view: row stride `stride`
        np.testing.assert_array_equal(dump(c), oracle.correlate(full[:, :n]))
    finally:
        c.close()


def test_narrow_batch_of_channels(X):
    # 64 channels of N = 64, T = 4096 in one batched call and as a prepared
    # batch launched twice (accumulating): every channel against the oracle
    chans, t = 64, 4096
    xs = synth.uniform_bytes(64, t * chans, seed=4300).reshape(chans, t, 64)
    c = X.Correlator(64, chans)
    try:
        dev = gpu(xs)
        jobs = [(c, k, dev[k]) for k in range(chans)]
        X.correlate_batch(jobs)
        want = [oracle.correlate(xs[k]) for k in range(chans)]
        for k in range(chans):
            np.testing.assert_array_equal(dump(c, k), want[k])
        b = X.Batch(jobs)
        b.launch()
        b.launch()
        torch.cuda.synchronize()
        assert b.check() == X.XENG_OK
        for k in range(chans):
            np.testing.assert_array_equal(dump(c, k), 2 * want[k])
        b.close()
    finally:
        c.close()


def test_narrow_wide_and_general_jobs_in_one_batch(X):
    # one call, three kernels: narrow (N = 16, 64), wide (N = 256), general
    # (N = 40: not a multiple of 16)
    shapes = [(16, 500), (64, 3000), (256, 700), (40, 333), (64, 1)]
    xs = [synth.uniform_bytes(n, t, seed=4400 + i) for i, (n, t) in enumerate(shapes)]
    cs = [X.Correlator(n, 1) for n, _ in shapes]
    try:
        X.correlate_batch([(c, 0, gpu(x)) for c, x in zip(cs, xs)])
        for c, x in zip(cs, xs):
            np.testing.assert_array_equal(dump(c), oracle.correlate(x))
    finally:
        for c in cs:
            c.close()


def test_narrow_equals_general_kernel(X):
    # the same job through the general kernel (forced) gives the same words
    n, t = 48, 2500
    x = synth.uniform_bytes(n, t, seed=4500)
    outs = []
    for kern in (X.XENG_KERNEL_AUTO, X.XENG_KERNEL_GENERAL):
        c = X.Correlator(n, 1)
        try:
            X.set_tuning(0, 0, kern)
            c.correlate(0, gpu(x))
            outs.append(dump(c))
        finally:
            X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
            c.close()
    np.testing.assert_array_equal(outs[0], outs[1])
