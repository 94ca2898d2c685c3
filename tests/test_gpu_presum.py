"""GPU parity of the unsigned-nibble form with pre-sums
(xeng_correlate_presum): every visibility against the oracle -- small and
ragged shapes on the wide kernel's unsigned instance (N a multiple of 16)
and on the general kernel's, the pre-sums of aligned rows (16-byte loads,
ragged column blocks and row slices) and of other arrays, both nibble
orders, unaligned arrays, pieces split at the
unsigned form's register bound, accumulation with the other kernels in one
slot, the correction applied once per dump (plain and batched exports, a
dump without reset, a reset that discards it), the full integration bound
where the unsigned sums pass int32, and the full-size N=2048 channel
against the oracle's recorded digest."""
import numpy as np
import pytest

import oracle
import oracle.presum as OP
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


def run(X, x, re_low=False):
    c = X.Correlator(x.shape[1], 1, re_low=re_low)
    c.correlate_presum(0, gpu(x))
    v = c.dump(0).cpu().numpy().astype(np.int64)
    c.close()
    return v


@pytest.mark.parametrize("n,t", [(1, 1), (2, 33), (5, 64), (16, 5), (48, 1000), (64, 4096), (100, 1000),
                                 (128, 129), (129, 300), (256, 65), (272, 300), (513, 129), (1000, 777),
                                 (32, 70001)])
def test_presum_matches_oracle(X, n, t):
    print(f"presum n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=[41, n, t])
    got = run(X, x)
    np.testing.assert_array_equal(got, oracle.correlate(x))
    np.testing.assert_array_equal(got, OP.correlate_presum(x))


def test_presum_re_low_and_unaligned(X):
    x = synth.uniform_bytes(70, 300, seed=42)
    np.testing.assert_array_equal(run(X, x, re_low=True), oracle.correlate(x, re_low=True))
    big = synth.uniform_bytes(105, 200, seed=43)
    c = X.Correlator(100, 1)
    c.correlate_presum(0, gpu(big)[:, 3:103])
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(big[:, 3:103]))
    c.close()


def test_presum_pieces_past_register_bound(X):
    # T = 600,000 > 2^19: every tile cut into pieces; extreme nibbles
    # maximise the unsigned sums
    n, t = 64, 600_000
    rng = np.random.default_rng(44)
    x = rng.choice(np.array([0x00, 0x0F, 0xF0, 0xFF, 0x88], dtype=np.uint8), size=(t, n))
    print(f"presum long pieces n={n} t={t}", flush=True)
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


def test_presum_mixed_with_other_kernels(X):
    n = 512
    xs = [synth.uniform_bytes(n, t, seed=[45, t]) for t in (300, 1000, 77)]
    c = X.Correlator(n, 1)
    c.correlate(0, gpu(xs[0]))                  # wide kernel
    c.correlate_presum(0, gpu(xs[1]))           # unsigned form
    c.correlate(0, gpu(xs[2]))
    assert c.samples_integrated(0) == 1377
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(np.concatenate(xs)))
    c.close()


def test_presum_at_the_integration_bound(X):
    # every sample 7+7j (u = 15): the unsigned sums reach 450 T, past int32,
    # and the corrections bring every pair back to Re = 98 T, Im = 0
    n = 64
    tmax = X.max_integration()
    chunk = 1 << 21
    ones = torch.full((chunk, n), 0xFF, dtype=torch.uint8, device="cuda")
    c = X.Correlator(n, 1)
    done = 0
    while done < tmax:
        k = min(chunk, tmax - done)
        c.correlate_presum(0, ones[:k])
        done += k
    v = c.dump(0).cpu().numpy().astype(np.int64)
    assert (v[:, 0] == 98 * tmax).all() and not v[:, 1].any()
    c.close()


def test_presum_full_size_digest(X):
    import parity_util as pu
    x = pu.fc.channel_n2048()
    print("presum full size n=2048 t=32768", flush=True)
    c = X.Correlator(2048, 1)
    c.correlate_presum(0, gpu(x))
    pu.assert_matches_oracle_digest("channel_n2048_t32768", c.dump(0), x)
    c.close()


def test_presum_wide_and_general_kernels_agree(X):
    # N a multiple of 16, contiguous: the wide kernel's unsigned instance;
    # forcing the general kernel gives the same words, both equal to the
    # oracle (rows past a piece's end read the unsigned zero sample)
    n, t = 256, 5000
    x = synth.uniform_bytes(n, t, seed=47)
    outs = []
    for kern in (X.XENG_KERNEL_AUTO, X.XENG_KERNEL_GENERAL):
        c = X.Correlator(n, 1)
        try:
            X.set_tuning(0, 0, kern)
            c.correlate_presum(0, gpu(x))
            outs.append(c.dump(0).cpu().numpy().astype(np.int64))
        finally:
            X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
            c.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], oracle.correlate(x))


def test_presum_wide_re_low(X):
    x = synth.uniform_bytes(128, 1000, seed=48)
    np.testing.assert_array_equal(run(X, x, re_low=True), oracle.correlate(x, re_low=True))


def test_presum_correction_applied_once_per_dump(X):
    # the correction of several unsigned-form calls (the wide kernel's, the
    # general kernel's through an unaligned view, and a signed call between
    # them) is applied once, before the dump; a dump without reset applies
    # it for good and later calls start a new one
    n = 256
    xs = [synth.uniform_bytes(n, t, seed=[49, t]) for t in (700, 300, 900, 500)]
    c = X.Correlator(n, 1)
    try:
        c.correlate_presum(0, gpu(xs[0]))                          # wide
        full = np.zeros((xs[1].shape[0], n + 3), dtype=np.uint8)
        full[:, 3:] = xs[1]
        c.correlate_presum(0, gpu(full)[:, 3:])                    # general, pre-sum pass
        c.correlate(0, gpu(xs[2]))                                  # signed
        got = c.dump(0, reset=False).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(got, oracle.correlate(np.concatenate(xs[:3])))
        c.correlate_presum(0, gpu(xs[3]))
        got = c.dump(0).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(got, oracle.correlate(np.concatenate(xs)))
        c.correlate(0, gpu(xs[0]))                                  # after the reset: no correction left
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(xs[0]))
    finally:
        c.close()


def test_presum_reset_discards_pending_correction(X):
    n = 128
    x1 = synth.uniform_bytes(n, 400, seed=50)
    x2 = synth.uniform_bytes(n, 300, seed=51)
    c = X.Correlator(n, 1)
    try:
        c.correlate_presum(0, gpu(x1))
        c.reset(0)
        c.correlate(0, gpu(x2))
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(x2))
    finally:
        c.close()


def test_presum_pending_corrections_in_a_batched_dump(X):
    # two contexts, three slots, pending corrections on two of them: one
    # batched export applies each before its slot is read
    a, b = X.Correlator(256, 2), X.Correlator(96, 1)
    xa0 = synth.uniform_bytes(256, 600, seed=52)
    xa1 = synth.uniform_bytes(256, 350, seed=53)
    xb = synth.uniform_bytes(96, 800, seed=54)
    try:
        a.correlate_presum(0, gpu(xa0))
        a.correlate(1, gpu(xa1))
        b.correlate_presum(0, gpu(xb))
        b.correlate_presum(0, gpu(xb))
        outs = X.dump_batch([(a, 0), (a, 1), (b, 0)])
        np.testing.assert_array_equal(outs[0].cpu().numpy().astype(np.int64), oracle.correlate(xa0))
        np.testing.assert_array_equal(outs[1].cpu().numpy().astype(np.int64), oracle.correlate(xa1))
        np.testing.assert_array_equal(outs[2].cpu().numpy().astype(np.int64),
                                      oracle.correlate(np.concatenate([xb, xb])))
    finally:
        a.close()
        b.close()


def test_presum_exports_in_a_row(X):
    # resetting exports apply the correction in their own kernels and switch
    # the slot between its two pre-sum buffers (clearing the one the next
    # calls use): four exports in a row, each of a different mix of calls,
    # FP8 included, every one against the oracle
    n = 192
    xs = [synth.uniform_bytes(n, t, seed=[55, t]) for t in (640, 330, 700, 257, 901, 64)]
    c = X.Correlator(n, 1)
    try:
        c.correlate_presum(0, gpu(xs[0]))
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(xs[0]))
        c.correlate_presum(0, gpu(xs[1]))
        c.correlate_presum(0, gpu(xs[2]))
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64),
                                      oracle.correlate(np.concatenate(xs[1:3])))
        c.correlate(0, gpu(xs[3]))
        X.set_tuning(0, 0, X.XENG_KERNEL_FP8)
        try:
            c.correlate(0, gpu(xs[4]))                                      # FP8: the unsigned form
        finally:
            X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64),
                                      oracle.correlate(np.concatenate(xs[3:5])))
        c.correlate_presum(0, gpu(xs[5]))
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(xs[5]))
    finally:
        c.close()
