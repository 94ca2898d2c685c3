"""GPU parity of phased-array beamforming (xeng_beamform): exact int32
beams and the 8-bit export, bit for bit against the oracle (oracle/beams.py)
-- ragged time and input counts, up to 16 beams, inputs past one LDS chunk,
both nibble orders, unaligned arrays, a coherent rank-1 closed form and the
full-size N=2048, T=32768, 10-beam workload."""
import ctypes

import numpy as np
import pytest

import oracle.beams as OB
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


@pytest.mark.parametrize("n,t,b", [(1, 1, 1), (16, 63, 10), (100, 65, 3), (256, 64, 16), (2048, 1000, 10),
                                   (3000, 129, 7), (4100, 70, 16), (48, 4096, 10)])
def test_beams_match_oracle(X, n, t, b):
    print(f"beamform n={n} t={t} beams={b}", flush=True)
    x = synth.uniform_bytes(n, t, seed=[61, n, t])
    w = synth.beam_weights(b, n, seed=[62, n])
    want = OB.beamform(x, w)
    got = X.beamform(gpu(x), w).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, want)
    for shift in (0, 5, 12):
        q = X.beamform(gpu(x), w, shift=shift).cpu().numpy()
        np.testing.assert_array_equal(q, OB.quantize(want, shift))


def test_beams_re_low_unaligned_and_extreme_weights(X):
    x = synth.uniform_bytes(70, 300, seed=63)
    w = np.random.default_rng(64).integers(-127, 128, size=(16, 70, 2)).astype(np.int8)
    w[3] = 127
    w[4] = -127
    swapped = ((x & 15) << 4) | (x >> 4)
    np.testing.assert_array_equal(X.beamform(gpu(swapped), w, re_low=True).cpu().numpy(), OB.beamform(x, w))
    big = synth.uniform_bytes(77, 300, seed=65)
    view = gpu(big)[:, 5:75]
    np.testing.assert_array_equal(X.beamform(view, w).cpu().numpy(), OB.beamform(big[:, 5:75], w))


def test_beams_rank1_coherent_closed_form(X):
    n, t = 2048, 256
    x, g_re, g_im = synth.rank1_tone(n, t, seed=66)
    w = np.stack([g_re, -g_im], axis=-1)[None].astype(np.int8)      # conj(g_i)
    y = X.beamform(gpu(x), w).cpu().numpy()
    p = int((g_re.astype(np.int64) ** 2 + g_im.astype(np.int64) ** 2).sum())
    rot = {0: (p, 0), 1: (0, p), 2: (-p, 0), 3: (0, -p)}
    for s in range(t):
        assert tuple(y[s, 0]) == rot[s % 4]


def test_beam_set_weights_and_argument_errors(X):
    # a beam set keeps its weights on the device; replacing them applies to
    # later calls on the stream
    n, t = 300, 500
    x = synth.uniform_bytes(n, t, seed=67)
    w1 = synth.beam_weights(10, n, seed=68)
    w2 = synth.beam_weights(10, n, seed=69)
    bm = X.Beams(w1)
    xd = gpu(x)
    y1 = bm.form(xd)
    bm.set_weights(w2)
    y2 = bm.form(xd)
    np.testing.assert_array_equal(y1.cpu().numpy(), OB.beamform(x, w1))
    np.testing.assert_array_equal(y2.cpu().numpy(), OB.beamform(x, w2))
    bad = w2.copy()
    bad[4, 7, 1] = -128                                              # outside [-127, 127]
    with pytest.raises(X.XengError) as e:
        bm.set_weights(bad)
    assert e.value.status == X.XENG_EINVAL
    np.testing.assert_array_equal(bm.form(xd).cpu().numpy(), OB.beamform(x, w2))   # unchanged
    bm.close()
    L = X.lib()
    h = ctypes.c_void_p()
    assert L.xeng_beams_create(n, 10, 0, 0, bad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == X.XENG_EINVAL
    w17 = np.zeros((17, n, 2), dtype=np.int8)
    assert L.xeng_beams_create(n, 17, 0, 0, w17.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == X.XENG_EINVAL
    bm = X.Beams(w1)
    out = torch.zeros((t, 10, 2), dtype=torch.int32, device="cuda")
    assert L.xeng_beamform(bm._h, ctypes.c_void_p(xd.data_ptr()), t, n, 25, ctypes.c_void_p(out.data_ptr()),
                           None) == X.XENG_EINVAL
    assert L.xeng_beamform(bm._h, ctypes.c_void_p(xd.data_ptr()), t, n - 1, -1, ctypes.c_void_p(out.data_ptr()),
                           None) == X.XENG_EINVAL
    bm.close()


def test_beams_full_size(X):
    n, t, b = 2048, 32768, 10
    print("beamform full size", flush=True)
    x = synth.chime_channel(n, t, seed=2)
    w = synth.beam_weights(b, n, seed=8)
    want = OB.beamform(x, w)
    got = X.beamform(gpu(x), w).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, want)
    q = X.beamform(gpu(x), w, shift=8).cpu().numpy()
    np.testing.assert_array_equal(q, OB.quantize(want, 8))
