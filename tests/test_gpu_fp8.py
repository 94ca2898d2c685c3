"""GPU parity of the exact FP8 paths (XENG_KERNEL_FP8).  Arrays the DMA
kernel reads in place take the wide kernel's FP8 instance of the unsigned
form: the stored nibbles are E4M3 codes as they are, fp32 sums stay exact
below 2^24 over pieces of at most 582 stages, and the pre-sum correction
brings them to the signed visibilities.  Batches and other arrays take the
general kernel's FP8 instance: every signed 4-bit value as its E4M3 code,
pieces below 2^17 samples.  Bit for bit against the CPU oracle: ragged
shapes, both nibble orders on both kernels, aligned and byte-addressed
rows, pieces at each kernel's exactness bound with extreme samples,
batches, a slot integrated by the int8 and the FP8 kernels in turn, and
the full-size N=2048 channel on both instances against the oracle's
recorded digest."""
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


@pytest.fixture
def fp8(X):
    X.set_tuning(0, 0, X.XENG_KERNEL_FP8)
    yield
    X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(X, x, re_low=False):
    c = X.Correlator(x.shape[1], 1, re_low=re_low)
    try:
        c.correlate(0, gpu(x))
        return c.dump(0).cpu().numpy().astype(np.int64)
    finally:
        c.close()


@pytest.mark.parametrize("n,t", [(1, 1), (5, 64), (16, 65), (64, 4096), (100, 1000), (128, 128), (129, 300),
                                 (256, 333), (300, 1000), (512, 2000)])
def test_fp8_matches_oracle(X, fp8, n, t):
    print(f"fp8 n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=5000 + n + t)
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


@pytest.mark.parametrize("n", [200, 256])
def test_fp8_re_low(X, fp8, n):
    # N = 200: the general kernel's instance; N = 256: the wide kernel's
    x = synth.uniform_bytes(n, 700, seed=5101)
    np.testing.assert_array_equal(run(X, x, re_low=True), oracle.correlate(x, re_low=True))


def test_fp8_byte_addressed_rows(X, fp8):
    # an odd row stride and base: the byte-load path of the kernel
    full = synth.uniform_bytes(101, 500, seed=5102)
    x = gpu(full)[:, 1:100]
    c = X.Correlator(99, 1)
    try:
        c.correlate(0, x)
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(full[:, 1:100]))
    finally:
        c.close()


def test_fp8_pieces_at_the_exactness_bound(X):
    # the general kernel's instance (rows at an odd byte offset): every
    # sample (-8, -8), so each pair adds 128 per sample.  One workgroup
    # takes the whole job in pieces of 2047 stages (131008 samples), whose
    # fp32 sums reach 128 * 131008 = 16,769,024, just under 2^24; every
    # piece but the last is exactly that long
    n, t = 128, 2 * 131008 + 4000
    full = np.zeros((t, n + 1), dtype=np.uint8)
    X.set_tuning(1, 1 << 20, X.XENG_KERNEL_FP8)
    c = X.Correlator(n, 1)
    try:
        c.correlate(0, gpu(full)[:, 1:])
        got = c.dump(0).cpu().numpy().astype(np.int64)
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
        c.close()
    assert (got[:, 0] == 128 * t).all()
    np.testing.assert_array_equal(got, oracle.correlate(full[:, 1:]))


@pytest.mark.parametrize("byte", [0xFF, 0xF0])
def test_fp8_wide_pieces_at_the_exactness_bound(X, byte):
    # the wide kernel's instance: every stored nibble pair (15, 15) makes
    # the unsigned real sums 450 per sample (or (15, 0): 225, with the
    # imaginary parts of mixed pairs at their extreme); pieces of 582
    # stages (37248 samples) reach 450 * 37248 = 16,761,600, just under
    # 2^24.  Columns of (15, 14) give odd sums per sample (435 against
    # (15, 15), 421 on their own diagonal), so pieces any longer would
    # round in fp32 and fail
    n, t = 256, 2 * 37248 + 4000
    x = np.full((t, n), byte, dtype=np.uint8)
    x[:, 1::3] = 0x0F
    x[:, 2::3] = 0xFE
    X.set_tuning(1, 1 << 20, X.XENG_KERNEL_FP8)
    try:
        got = run(X, x)
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
    np.testing.assert_array_equal(got, oracle.correlate(x))


def test_fp8_extreme_samples_split(X, fp8):
    rng = np.random.default_rng(18)
    n, t = 256, 140_000
    x = rng.choice(np.array([0x00, 0x0F, 0xF0, 0xFF, 0x80, 0x08, 0x77], dtype=np.uint8), size=(t, n))
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


def test_fp8_batch(X, fp8):
    shapes = [(64, 1000), (256, 700), (100, 333), (512, 129)]
    xs = [synth.uniform_bytes(n, t, seed=5200 + i) for i, (n, t) in enumerate(shapes)]
    cs = [X.Correlator(n, 1) for n, _ in shapes]
    try:
        X.correlate_batch([(c, 0, gpu(x)) for c, x in zip(cs, xs)])
        for c, x in zip(cs, xs):
            np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(x))
    finally:
        for c in cs:
            c.close()


def test_fp8_and_int8_on_one_slot(X):
    # the int8 kernels and the wide FP8 path store Im V_ij - S_j (the dump
    # removes S_j through the diagonal), the general FP8 instance Im V_ij
    # itself; a slot integrated by all of them in turn still exports exact
    # visibilities
    n, t = 256, 3000
    x = synth.uniform_bytes(n, t, seed=5300)
    c = X.Correlator(n, 1)
    try:
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
        c.correlate(0, gpu(x[:1000]))
        X.set_tuning(0, 0, X.XENG_KERNEL_FP8)
        c.correlate(0, gpu(x[1000:2200]))                                  # wide FP8
        full = np.zeros((400, n + 3), dtype=np.uint8)
        full[:, 3:] = x[2200:2600]
        c.correlate(0, gpu(full)[:, 3:])                                   # general FP8
        X.set_tuning(0, 0, X.XENG_KERNEL_GENERAL)
        c.correlate(0, gpu(x[2600:]))
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(x))
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
        c.close()


@pytest.mark.parametrize("path", ["wide", "general"])
def test_fp8_full_size_digest(X, fp8, path):
    # the N=2048, T=32768 channel on each FP8 instance (the general one
    # through a view at a one-byte offset), every pair against the oracle's
    # recorded digest
    import parity_util as pu
    x = pu.fc.channel_n2048()
    print(f"fp8 full size n=2048 t=32768 {path}", flush=True)
    c = X.Correlator(2048, 1)
    try:
        if path == "wide":
            c.correlate(0, gpu(x))
        else:
            full = np.zeros((x.shape[0], x.shape[1] + 1), dtype=np.uint8)
            full[:, 1:] = x
            c.correlate(0, gpu(full)[:, 1:])
        pu.assert_matches_oracle_digest("channel_n2048_t32768", c.dump(0), x)
    finally:
        c.close()


def test_fp8_batches_eager_and_prepared(X, fp8):
    # eager batches take the wide kernel's FP8 instance for the arrays it
    # reads in place (N = 128, 96), whose pre-sums add up in the slots over
    # two calls and are corrected at a batched export, and the general
    # kernel's for the rest (N = 100); prepared batches take the general
    # kernel's instance throughout
    shapes = [(128, 900), (96, 333), (100, 500)]
    xs = [synth.uniform_bytes(n, t, seed=5400 + i) for i, (n, t) in enumerate(shapes)]
    refs = [oracle.correlate(np.concatenate([x, x])) for x in xs]
    cs = [X.Correlator(n, 1) for n, _ in shapes]
    bufs = [gpu(x) for x in xs]
    try:
        X.correlate_batch([(c, 0, b) for c, b in zip(cs, bufs)])
        X.correlate_batch([(c, 0, b) for c, b in zip(cs, bufs)])
        outs = X.dump_batch([(c, 0) for c in cs])
        for o, r in zip(outs, refs):
            np.testing.assert_array_equal(o.cpu().numpy().astype(np.int64), r)
        b = X.Batch([(c, 0, t) for c, t in zip(cs, bufs)])
        try:
            b.launch()
            b.launch()
            assert b.check() == X.XENG_OK
            for c, r in zip(cs, refs):
                np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), r)
        finally:
            b.close()
    finally:
        for c in cs:
            c.close()
