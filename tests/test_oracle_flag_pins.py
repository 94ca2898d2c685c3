"""Pins for the flag-aware oracle (oracle/flags.py): the RFI-excision
estimator against a hand-worked example and closed forms, and the
flag-aware correlation against per-sample Python loops, extreme flag
patterns and additivity in time.  ``test_flag_pins_catch_planted_mistakes``
plants typical mistakes in a copy of the oracle's source and checks that
the battery fails each one."""
import os
import types

import numpy as np
import pytest

import oracle
import oracle.flags as OF
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    rows = {}
    with open(os.path.join(GOLDEN, "sk_example.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, *v = line.split("|")
                rows[k] = v
    return rows


def _enc(re, im):
    return synth.encode(np.asarray(re), np.asarray(im))


# ---------------------------------------------------------------------------
# Battery: each pin takes the module under test (the oracle or a mutant).
# ---------------------------------------------------------------------------

def pin_sk_worked_example(of):
    g = _golden()
    x = np.array([[int(h, 16) for h in r.split()] for r in g["samples"]], dtype=np.uint8)
    re, im = oracle.decode(x)
    p = re * re + im * im
    for i, want in enumerate(g["sk"]):
        s1, s2 = int(p[:, i].sum()), int((p[:, i] ** 2).sum())
        got = of.sk_value(s1, s2, 4)
        if want == "-":
            assert got is None
        else:
            a, b = map(int, want.split("/"))
            assert got is not None and got[0] * b == a * got[1], (i, got, want)
    f1 = of.sk_flags(x, block_len=4, lo_num=625, hi_num=1375, den=1000)
    np.testing.assert_array_equal(f1[0], [int(v) for v in g["flags_625_1375"][0].split()])
    f2 = of.sk_flags(x, block_len=4, lo_num=600, hi_num=4000, den=1000)
    np.testing.assert_array_equal(f2[0], [int(v) for v in g["flags_600_4000"][0].split()])


def pin_sk_two_level_closed_form(of):
    # powers alternating a, b over an even block: M S2 / S1^2 = 2 (a^2 + b^2) / (a + b)^2,
    # so SK = (M + 1) / (M - 1) * (a - b)^2 / (a + b)^2
    cases = [((1, 0), (2, 0)), ((1, 1), (3, 0)), ((0, 2), (7, 7)), ((5, 5), (-5, -5))]
    for m in (2, 4, 16, 256):
        for (ra, ia), (rb, ib) in cases:
            re = np.array([ra, rb] * (m // 2))
            im = np.array([ia, ib] * (m // 2))
            x = _enc(re, im)[:, None]
            a, b = ra * ra + ia * ia, rb * rb + ib * ib
            s1, s2 = int(m // 2 * (a + b)), int(m // 2 * (a * a + b * b))
            num, den = of.sk_value(s1, s2, m)
            assert num * (m - 1) * (a + b) ** 2 == den * (m + 1) * (a - b) ** 2
            # a threshold just above and just below the exact value
            if a != b:
                sk_n, sk_d = (m + 1) * (a - b) ** 2, (m - 1) * (a + b) ** 2
                assert of.sk_flags(x, block_len=m, lo_num=sk_n + 1, hi_num=10 ** 9, den=sk_d)[0, 0] == 1
                assert of.sk_flags(x, block_len=m, lo_num=sk_n, hi_num=10 ** 9, den=sk_d)[0, 0] == 0
                assert of.sk_flags(x, block_len=m, lo_num=0, hi_num=sk_n - 1, den=sk_d)[0, 0] == 1
                assert of.sk_flags(x, block_len=m, lo_num=0, hi_num=sk_n, den=sk_d)[0, 0] == 0


def pin_sk_constant_power_and_no_power(of):
    t = 1000
    x, _, _ = synth.rank1_tone(3, t, seed=3)           # |x_i(t)| constant in t
    f = of.sk_flags(x, block_len=100, lo_num=1, hi_num=5000, den=1000)
    assert f.shape == (10, 3) and f.all()               # SK = 0 < 0.001
    assert not of.sk_flags(x, block_len=100, lo_num=0, hi_num=5000, den=1000).any()
    z = np.full((300, 2), 0x88, dtype=np.uint8)         # no power at all: flagged
    assert of.sk_flags(z, block_len=64, lo_num=0, hi_num=10 ** 6, den=1).all()
    # a last block of one sample is never flagged (M - 1 = 0)
    y = np.concatenate([x[:100], np.full((1, 3), 0x88, dtype=np.uint8)])
    f = of.sk_flags(y, block_len=100, lo_num=1, hi_num=5000, den=1000)
    assert f.shape == (2, 3) and f[0].all() and not f[1].any()


def pin_sk_gaussian_noise_mostly_kept(of):
    x = synth.gaussian_bytes(64, 256 * 40, seed=5)
    f = of.sk_flags(x, block_len=256)                    # 1 +- 0.375, about 3 sigma at M = 256
    assert f.mean() < 0.03, f.mean()


def pin_counts_and_vis_brute_force(of):
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 5))
        t = int(rng.integers(0, 13))
        bl = int(rng.integers(1, 6))
        x = rng.integers(0, 256, size=(t, n), dtype=np.uint8)
        nb = of.n_blocks(t, bl)
        fl = (rng.random((nb, n)) < 0.4).astype(np.uint8)
        vis, cnt = of.correlate_flagged(x, fl, bl)
        assert list(cnt) == of.counts_python(fl, bl, t, n)
        k = 0
        for i in range(n):
            for j in range(i, n):
                acc = 0j
                for s in range(t):
                    if fl[s // bl][i] or fl[s // bl][j]:
                        continue
                    xi = complex((int(x[s, i]) >> 4) - 8, (int(x[s, i]) & 15) - 8)
                    xj = complex((int(x[s, j]) >> 4) - 8, (int(x[s, j]) & 15) - 8)
                    acc += xi * xj.conjugate()
                assert (vis[k, 0], vis[k, 1]) == (int(acc.real), int(acc.imag))
                k += 1


def pin_flag_extremes(of):
    x = synth.uniform_bytes(40, 1000, seed=12)
    bl = 64
    nb = of.n_blocks(1000, bl)
    vis, cnt = of.correlate_flagged(x, np.zeros((nb, 40), np.uint8), bl)
    np.testing.assert_array_equal(vis, oracle.correlate(x))
    assert (cnt == 1000).all()
    vis, cnt = of.correlate_flagged(x, np.ones((nb, 40), np.uint8), bl)
    assert not vis.any() and not cnt.any()
    fl = np.zeros((nb, 40), np.uint8)
    fl[:, 7] = 1                                         # input 7 flagged throughout
    fl[3, :] = 1                                         # block 3 flagged on every input
    vis, cnt = of.correlate_flagged(x, fl, bl)
    n = 40
    for i in range(n):
        for j in range(i, n):
            k = oracle.tri_index(i, j, n)
            if 7 in (i, j):
                assert cnt[k] == 0 and not vis[k].any()
            else:
                assert cnt[k] == 1000 - bl


def pin_additivity_at_block_boundaries(of):
    x = synth.uniform_bytes(30, 700, seed=13)
    bl = 50
    rng = np.random.default_rng(14)
    fl = (rng.random((of.n_blocks(700, bl), 30)) < 0.3).astype(np.uint8)
    vis, cnt = of.correlate_flagged(x, fl, bl)
    for cut in (50, 300, 650):
        a = of.correlate_flagged(x[:cut], fl[:cut // bl], bl)
        b = of.correlate_flagged(x[cut:], fl[cut // bl:], bl)
        np.testing.assert_array_equal(a[0] + b[0], vis)
        np.testing.assert_array_equal(a[1] + b[1], cnt)


PINS = [pin_sk_worked_example, pin_sk_two_level_closed_form, pin_sk_constant_power_and_no_power,
        pin_sk_gaussian_noise_mostly_kept, pin_counts_and_vis_brute_force, pin_flag_extremes,
        pin_additivity_at_block_boundaries]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_flag_pin(pin, oracle_lib):
    pin(OF)


def test_rfi_channel_cells_are_flagged(oracle_lib):
    # the generator's injected cells (constant-power carriers, impulsive and
    # broadband bursts) are flagged; the CHIME-shaped rest mostly is not
    n, t, bl = 64, 256 * 32, 256
    x = synth.rfi_channel(n, t, seed=6, block_len=bl, tone_frac=0.05, burst_frac=0.03, broadband_blocks=1)
    f = OF.sk_flags(x, block_len=bl)
    re, im = oracle.decode(x)
    p = (re * re + im * im).reshape(t // bl, bl, n)
    const = (p == p[:, :1, :]).all(axis=1)               # constant-power cells: the carriers
    spiky = (p == 0).sum(axis=1) >= bl - 4               # silenced cells with a few spikes
    assert const.sum() >= 0.04 * f.size and spiky.sum() >= 0.02 * f.size
    assert f[const].all() and f[spiky].all()
    assert f[~(const | spiky)].mean() < 0.03


MUTANTS = {
    "counts_or_instead_of_and": ("full = (w * lens[:, None]).T @ w", "full = ((1 - w) * lens[:, None]).T @ (1 - w)"),
    "block_index_off_by_one": ("rows = slice(b * block_len, min((b + 1) * block_len, t))",
                               "rows = slice(b * block_len + 1, min((b + 1) * block_len + 1, t))"),
    "sk_factor_inverted": ("return (m + 1) * (m * s2 - s1 * s1), (m - 1) * s1 * s1",
                           "return (m - 1) * (m * s2 - s1 * s1), (m + 1) * s1 * s1"),
    "sk_threshold_not_strict": ("return num * den < lo_num * dd or num * den > hi_num * dd",
                                "return num * den <= lo_num * dd or num * den > hi_num * dd"),
    "no_power_kept": ("    if v is None:\n        return True", "    if v is None:\n        return False"),
    "last_block_full_length": ("lens[-1] = n_samples - (nb - 1) * block_len", "lens[-1] = block_len"),
    "mask_wrong_axis": ("s[rows, flags[b] != 0] = 0x88", "s[rows, flags[b] == 0] = 0x88"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_flag_pins_catch_planted_mistakes(name, oracle_lib):
    src = open(OF.__file__).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._flags_mutant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            failed.append(pin.__name__)
        except Exception as e:                   # a mutant may also crash a pin
            failed.append(f"{pin.__name__}: {type(e).__name__}")
    assert failed, f"no pin caught mutant {name}"
