"""Pins for the pre-sum oracle (oracle/presum.py): the unsigned products
plus O(N) corrections equal the definition written out (the C oracle, itself
pinned in test_oracle_pins.py) and Python complex arithmetic on tiny inputs,
and give the closed forms of extreme inputs; planted mistakes in its source
(a dropped correction, a wrong sign or factor, swapped nibbles) are caught."""
import types

import numpy as np
import pytest

import oracle
import oracle.presum as OP
import synth


def pin_matches_definition(op):
    for seed, (n, t) in enumerate([(1, 1), (2, 5), (7, 100), (33, 257), (64, 1000)]):
        x = synth.uniform_bytes(n, t, seed=[31, seed])
        np.testing.assert_array_equal(op.correlate_presum(x), oracle.correlate(x))
        np.testing.assert_array_equal(op.correlate_presum(x, re_low=True), oracle.correlate(x, re_low=True))


def pin_python_complex_tiny(op):
    rng = np.random.default_rng(32)
    for _ in range(20):
        n, t = int(rng.integers(1, 4)), int(rng.integers(0, 7))
        x = rng.integers(0, 256, size=(t, n), dtype=np.uint8)
        got = op.correlate_presum(x)
        want = oracle.correlate_python(x, n_inputs=n)
        assert [tuple(map(int, r)) for r in got] == want


def pin_extremes(op):
    t = 1000
    lo = np.zeros((t, 3), dtype=np.uint8)            # u = 0: x = -8-8j everywhere
    v = op.correlate_presum(lo)
    assert (v[:, 0] == 128 * t).all() and not v[:, 1].any()
    hi = np.full((t, 3), 0xFF, dtype=np.uint8)       # u = 15: x = 7+7j
    v = op.correlate_presum(hi)
    assert (v[:, 0] == 98 * t).all() and not v[:, 1].any()
    z = np.full((t, 3), 0x88, dtype=np.uint8)        # u = 8: x = 0
    assert not op.correlate_presum(z).any()
    # pre-sums of the zero sample: 8 T per input
    sr, si = op.presums(z)
    assert (sr == 8 * t).all() and (si == 8 * t).all()


def pin_rank1_tone(op):
    x, g_re, g_im = synth.rank1_tone(20, 400, seed=33)
    v = op.correlate_presum(x)
    iu, ju = np.triu_indices(20)
    np.testing.assert_array_equal(v[:, 0], 400 * (g_re[iu] * g_re[ju] + g_im[iu] * g_im[ju]))
    np.testing.assert_array_equal(v[:, 1], 400 * (g_im[iu] * g_re[ju] - g_re[iu] * g_im[ju]))


PINS = [pin_matches_definition, pin_python_complex_tiny, pin_extremes, pin_rank1_tone]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_presum_pin(pin, oracle_lib):
    pin(OP)


MUTANTS = {
    "dropped_constant": ("+ 128 * t", ""),
    "single_constant": ("+ 128 * t", "+ 64 * t"),
    "im_correction_sign": ("im = uim + 8 * (sr - si)[:, None] - 8 * (sr - si)[None, :]",
                           "im = uim - 8 * (sr - si)[:, None] + 8 * (sr - si)[None, :]"),
    "re_correction_factor": ("re = ure - 8 * (sr + si)[:, None]", "re = ure - 4 * (sr + si)[:, None]"),
    "nibbles_swapped": ("return (lo, hi) if re_low else (hi, lo)", "return (hi, lo) if re_low else (lo, hi)"),
    "im_products_transposed": ("ui.T @ ur - ur.T @ ui", "ur.T @ ui - ui.T @ ur"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_presum_pins_catch_planted_mistakes(name, oracle_lib):
    src = open(OP.__file__).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._presum_mutant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutant {name}"
