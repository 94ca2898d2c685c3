"""Pins for the beamforming oracle (oracle/beams.py): Python complex
arithmetic on tiny inputs, a single-input beam reproducing that input, a
rank-1 tone summed coherently by conjugate weights (closed form), linearity
in the weights, and the rounding of the 8-bit export at exact halves; a
planted mistake in its source (a dropped or sign-flipped cross term,
conjugated weights, rounding away from even) is caught."""
import types

import numpy as np
import pytest

import oracle.beams as OB
import synth


def pin_python_complex_tiny(ob):
    rng = np.random.default_rng(51)
    for _ in range(20):
        n, t, b = int(rng.integers(1, 5)), int(rng.integers(0, 6)), int(rng.integers(1, 4))
        x = rng.integers(0, 256, size=(t, n), dtype=np.uint8)
        w = rng.integers(-127, 128, size=(b, n, 2)).astype(np.int8)
        got = ob.beamform(x, w, n)
        assert [[tuple(map(int, v)) for v in row] for row in got] == ob.beamform_python(x, w, n)


def pin_single_input_beam(ob):
    x = synth.uniform_bytes(5, 200, seed=52)
    w = np.zeros((3, 5, 2), dtype=np.int8)
    w[0, 2] = (1, 0)              # beam 0 = input 2
    w[1, 4] = (0, 1)              # beam 1 = j * input 4
    y = ob.beamform(x, w)
    re = (x.astype(np.int64) >> 4) - 8
    im = (x.astype(np.int64) & 15) - 8
    np.testing.assert_array_equal(y[:, 0, 0], re[:, 2])
    np.testing.assert_array_equal(y[:, 0, 1], im[:, 2])
    np.testing.assert_array_equal(y[:, 1, 0], -im[:, 4])
    np.testing.assert_array_equal(y[:, 1, 1], re[:, 4])
    assert not y[:, 2].any()


def pin_rank1_coherent_sum(ob):
    # x_i(t) = g_i j^t with conjugate weights conj(g_i): y(t) = j^t sum |g_i|^2
    n, t = 30, 64
    x, g_re, g_im = synth.rank1_tone(n, t, seed=53)
    w = np.stack([np.stack([g_re, -g_im], axis=-1)], axis=0).astype(np.int8)
    y = ob.beamform(x, w)
    p = int((g_re.astype(np.int64) ** 2 + g_im.astype(np.int64) ** 2).sum())
    want = {0: (p, 0), 1: (0, p), 2: (-p, 0), 3: (0, -p)}
    for s in range(t):
        assert tuple(y[s, 0]) == want[s % 4]


def pin_linear_in_weights(ob):
    x = synth.uniform_bytes(40, 100, seed=54)
    rng = np.random.default_rng(55)
    a = rng.integers(-60, 61, size=(2, 40, 2)).astype(np.int8)
    b = rng.integers(-60, 61, size=(2, 40, 2)).astype(np.int8)
    np.testing.assert_array_equal(ob.beamform(x, a) + ob.beamform(x, b), ob.beamform(x, (a + b).astype(np.int8)))


def pin_quantize_halves(ob):
    v = np.array([0, 1, 2, 3, 4, 5, 6, 7, -1, -2, -3, -4, -5, -6, 1000000, -1000000], dtype=np.int64)
    # shift 1: v / 2 = 0, .5, 1, 1.5, 2, 2.5, 3, 3.5 -> 0 0 1 2 2 2 3 4 ; negatives mirror
    want = [0, 0, 1, 2, 2, 2, 3, 4, 0, -1, -2, -2, -2, -3, 127, -127]
    np.testing.assert_array_equal(ob.quantize(v, 1), want)
    np.testing.assert_array_equal(ob.quantize(np.array([12, 20, 28, -12]), 3), [2, 2, 4, -2])   # 1.5 2.5 3.5 -1.5
    np.testing.assert_array_equal(ob.quantize(np.array([127, 128, -127, -128]), 0), [127, 127, -127, -127])


PINS = [pin_python_complex_tiny, pin_single_input_beam, pin_rank1_coherent_sum, pin_linear_in_weights,
        pin_quantize_halves]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_beam_pin(pin):
    pin(OB)


MUTANTS = {
    "cross_term_sign": ("yr = xr @ wr.T - xi @ wi.T", "yr = xr @ wr.T + xi @ wi.T"),
    "dropped_cross_term": ("yi = xr @ wi.T + xi @ wr.T", "yi = xr @ wi.T"),
    "conjugated_weights": ("wr, wi = w[:, :, 0], w[:, :, 1]", "wr, wi = w[:, :, 0], -w[:, :, 1]"),
    "round_half_up": ("round(Fraction(int(v), 1 << shift))", "(Fraction(int(v), 1 << shift) + Fraction(1, 2)).__floor__()"),
    "truncate": ("round(Fraction(int(v), 1 << shift))", "int(Fraction(int(v), 1 << shift))"),
    "clip_128": ("max(-127, min(127,", "max(-128, min(128,"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_beam_pins_catch_planted_mistakes(name):
    src = open(OB.__file__).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._beams_mutant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, OverflowError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutant {name}"
