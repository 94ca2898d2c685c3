"""The allocation-free entry point (xeng_correlate_static), called through
the C ABI: its output equals xeng_correlate's, bit for bit, on two calls in
a row on one GPU (the second smaller, reusing the fixed plan array), for the
wide kernel, the 128 x 128 kernel and an accumulating slot."""
import ctypes

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


def both_paths(X, n, xs):
    """Correlate each array of `xs` (a call per array, into one slot) with
    xeng_correlate_static and with xeng_correlate; return both exports."""
    L = X.lib()
    outs = []
    for fn in (L.xeng_correlate_static, L.xeng_correlate):
        c = X.Correlator(n, 1)
        keep = []
        for x in xs:
            d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
            keep.append(d)
            rc = fn(c.handle, 0, ctypes.c_void_p(d.data_ptr()), d.shape[0], d.stride(0),
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert rc == X.XENG_OK, X.strerror(rc)
        assert c.samples_integrated(0) == sum(x.shape[0] for x in xs)
        outs.append(c.dump(0).cpu().numpy().astype(np.int64))
        c.close()
    return outs


@pytest.mark.parametrize("n", [2048, 512, 100])
def test_static_matches_correlate_two_calls(X, n):
    # first call larger than the second: the second call's plan overwrites
    # the first's in the fixed array while the first may still be queued
    L = X.lib()
    big = synth.chime_channel(n, 8192 + 37, seed=[71, n])
    small = synth.uniform_bytes(n, 700, seed=[72, n])
    print(f"static path n={n}: two calls", flush=True)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for x in (big, small):
        d = torch.from_numpy(x).cuda()
        c = X.Correlator(n, 1)
        ref_c = X.Correlator(n, 1)
        assert L.xeng_correlate_static(c.handle, 0, ctypes.c_void_p(d.data_ptr()), x.shape[0], n,
                                       stream) == X.XENG_OK
        assert L.xeng_correlate(ref_c.handle, 0, ctypes.c_void_p(d.data_ptr()), x.shape[0], n,
                                stream) == X.XENG_OK
        got = c.dump(0).cpu().numpy().astype(np.int64)
        want = ref_c.dump(0).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(got, want)
        if x is small:
            np.testing.assert_array_equal(got, oracle.correlate(x))
        c.close()
        ref_c.close()


def test_static_accumulates_and_matches(X):
    # several calls into one slot, the later ones smaller (not a fresh slot)
    n = 512
    xs = [synth.uniform_bytes(n, t, seed=[73, t]) for t in (3000, 1000, 65, 1)]
    got, want = both_paths(X, n, xs)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(got, oracle.correlate(np.concatenate(xs)))


def test_static_rejects_plan_past_its_array(X):
    # N = 46337 (not a multiple of 16: 128 x 128 tiles, 363 per side) has
    # 66,066 tiles, more pieces than the 1 MiB array holds at any T: refused
    # with XENG_ENOMEM before anything is queued.  The samples are real
    # device memory of the full [T][N] shape all the same.
    L = X.lib()
    n, t = 46337, 64
    pieces = X.plan_inspect_static(n, t, 512, 4, wide=False)
    assert len(pieces) * 16 > (1 << 20)
    c = X.Correlator(n, 1)
    d = torch.full((t, n), 0x88, dtype=torch.uint8, device="cuda")
    rc = L.xeng_correlate_static(c.handle, 0, ctypes.c_void_p(d.data_ptr()), t, n, None)
    assert rc == X.XENG_ENOMEM
    assert c.samples_integrated(0) == 0
    assert L.xeng_correlate_static(c.handle, 0, ctypes.c_void_p(d.data_ptr()), 1, 0, None) == X.XENG_EINVAL
    c.close()
