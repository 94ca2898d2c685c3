"""The seeded input generators: deterministic, in range, shaped as stated."""
import numpy as np

import synth


def _parts(x):
    return (x >> 4).astype(int) - 8, (x & 15).astype(int) - 8


def test_deterministic_per_seed():
    a = synth.chime_channel(64, 300, seed=2)
    b = synth.chime_channel(64, 300, seed=2)
    c = synth.chime_channel(64, 300, seed=3)
    assert a.dtype == np.uint8 and a.shape == (300, 64)
    np.testing.assert_array_equal(a, b)
    assert (a != c).any()


def test_value_ranges():
    re, im = _parts(synth.chime_channel(128, 4096, seed=2))
    assert re.min() >= -7 and re.max() <= 7 and im.min() >= -7 and im.max() <= 7
    re, im = _parts(synth.gaussian_bytes(64, 2048, seed=4))
    assert re.min() >= -7 and im.max() <= 7
    re, im = _parts(synth.uniform_bytes(64, 4096, seed=1))
    assert re.min() == -8 and re.max() == 7 and im.min() == -8 and im.max() == 7


def test_chime_channel_statistics():
    # power 3^2 * (1 noise + 0.1 sky + 3 * 0.3^2 tones) = 12.3, plus rounding
    x = synth.chime_channel(256, 8192, seed=2)
    re, im = _parts(x)
    p = (re.astype(float) ** 2 + im.astype(float) ** 2).mean()
    assert 11.5 < p < 13.5
    z = re + 1j * im
    c = (z[:, 0] * np.conj(z[:, 1])).mean()          # common sky + tones correlate inputs
    assert abs(c) > 0.3


def test_flagging_and_batches():
    chans = synth.batched_channels(n_channels=3, n_inputs=128, t_lo=100, t_hi=300, seed=3)
    assert len(chans) == 3
    for x in chans:
        assert 100 <= x.shape[0] <= 300
        flagged = np.all(x == synth.gen.FLAG_BYTE, axis=0)
        assert flagged.sum() == round(0.05 * 128)
    subs = synth.subarray_batch(n_instances=5, n_choices=(16, 32), t_choices=(8, 16), seed=4)
    assert all(s.shape[1] in (16, 32) and s.shape[0] in (8, 16) for s in subs)


def test_encode_rejects_out_of_range():
    import pytest
    with pytest.raises(ValueError):
        synth.encode(np.array([8]), np.array([0]))


def test_rank1_tone_stays_in_range():
    x, g_re, g_im = synth.rank1_tone(30, 17, seed=1, quarter_turns=1)
    re, im = _parts(x)
    assert re.min() >= -7 and re.max() <= 7
    np.testing.assert_array_equal(re[0], g_re)
    np.testing.assert_array_equal(im[0], g_im)
    np.testing.assert_array_equal(re[1], -g_im)   # multiplied by j once
