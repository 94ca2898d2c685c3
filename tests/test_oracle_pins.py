"""Pins for the CPU oracle, checked against things other than itself.

Every check here is fixed by the paper or by mathematics: printed values
(golden files), brute force with Python complex numbers, a library complex
matrix product, closed forms (a rank-1 tone), invariants (Hermitian
symmetry, diagonal = power, additivity in time, conjugation symmetries) and
extreme inputs.  ``test_pins_catch_planted_mistakes`` plants typical
mistakes in a copy of the oracle's C source and checks that the battery
fails every one of them.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split("|"))
    return rows


def _x(b):
    """Reference decode of one byte as a Python complex (real = high nibble)."""
    return complex((b >> 4) - 8, (b & 15) - 8)


# ---------------------------------------------------------------------------
# Battery of pins; each takes a `corr(samples, **kw)` callable so that the
# same battery can be run against planted-mistake builds of the oracle.
# ---------------------------------------------------------------------------

def pin_worked_example(corr):
    rows = dict((r[0], r[1:]) for r in _read_rows("worked_example.txt"))
    samples = np.array([[int(h, 16) for h in r.split()] for r in rows["samples"]], dtype=np.uint8)
    expected = np.array([[int(v) for v in r.split()] for r in rows["expected"]], dtype=np.int64)
    np.testing.assert_array_equal(corr(samples), expected)


def pin_python_complex_tiny(corr):
    for seed in range(6):
        rng = _rng(seed)
        for n in (1, 2, 3, 4):
            for t in (0, 1, 2, 5, 8):
                x = rng.integers(0, 256, size=(t, n), dtype=np.uint8)
                got = corr(x)
                ref = np.array(oracle.correlate_python(x, n), dtype=np.int64).reshape(-1, 2)
                np.testing.assert_array_equal(got, ref)


def pin_exhaustive_byte_pairs(corr):
    # Inputs 0..255 carry every byte once at T=1 and inputs 256..511 repeat
    # them, so pairs (i, 256 + j) cover every ordered byte pair (i, j).
    x = np.concatenate([np.arange(256), np.arange(256)]).astype(np.uint8)[None, :]
    got = corr(x)
    n = 512
    xs = [_x(b) for b in range(256)]
    ref = np.array([[p.real, p.imag] for p in
                    (xs[a] * xs[b].conjugate() for a in range(256) for b in range(256))],
                   dtype=np.int64).reshape(256, 256, 2)
    i = np.arange(256)[:, None]
    j = 256 + np.arange(256)[None, :]
    k = i * n - i * (i - 1) // 2 + (j - i)
    np.testing.assert_array_equal(got[k], ref)


def pin_rank1_tone(corr):
    for qt in (0, 1, 2, 3):
        for n, t in ((5, 37), (16, 64)):
            x, g_re, g_im = synth.rank1_tone(n, t, seed=qt + n, quarter_turns=qt)
            got = corr(x)
            g = [complex(int(a), int(b)) for a, b in zip(g_re, g_im)]
            ref = [(t * g[i] * g[j].conjugate()) for i in range(n) for j in range(i, n)]
            ref = np.array([[int(v.real), int(v.imag)] for v in ref], dtype=np.int64)
            np.testing.assert_array_equal(got, ref)


def pin_diagonal_power(corr):
    x = synth.uniform_bytes(9, 300, seed=11)
    got = corr(x)
    n = 9
    for i in range(n):
        p = sum(abs(_x(int(b))) ** 2 for b in x[:, i])
        k = oracle.tri_index(i, i, n)
        assert got[k, 0] == int(round(p)) and got[k, 1] == 0


def pin_extremes(corr):
    t, n = 33, 6
    assert not corr(np.full((t, n), 0x88, np.uint8)).any()
    got = corr(np.zeros((t, n), np.uint8))          # every sample -8 - 8j
    assert (got[:, 0] == 128 * t).all() and (got[:, 1] == 0).all()


def pin_nibble_swap_is_conjugate(corr):
    x = synth.uniform_bytes(7, 50, seed=3)
    swapped = ((x << 4) | (x >> 4)).astype(np.uint8)
    a, b = corr(x), corr(swapped)
    np.testing.assert_array_equal(b[:, 0], a[:, 0])
    np.testing.assert_array_equal(b[:, 1], -a[:, 1])


def pin_numpy_matmul(corr):
    for (n, t, seed) in ((33, 257, 1), (70, 100, 2)):
        x = synth.uniform_bytes(n, t, seed=seed)
        np.testing.assert_array_equal(corr(x), oracle.correlate_numpy(x))


def pin_permutation(corr):
    n, t = 8, 40
    x = synth.uniform_bytes(n, t, seed=5)
    perm = _rng(6).permutation(n)
    a = corr(x)
    b = corr(x[:, perm])
    for i in range(n):
        for j in range(i, n):
            p, q = perm[i], perm[j]
            if p <= q:
                ref = a[oracle.tri_index(p, q, n)]
            else:
                ref = a[oracle.tri_index(q, p, n)] * np.array([1, -1])
            np.testing.assert_array_equal(b[oracle.tri_index(i, j, n)], ref)


PINS = [pin_worked_example, pin_python_complex_tiny, pin_exhaustive_byte_pairs,
        pin_rank1_tone, pin_diagonal_power, pin_extremes, pin_nibble_swap_is_conjugate,
        pin_numpy_matmul, pin_permutation]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin, oracle_lib):
    pin(lambda s, **kw: oracle.correlate(s, **kw))


# ---------------------------------------------------------------------------
# Invariants of the full-matrix and accumulation modes
# ---------------------------------------------------------------------------

def test_full_matrix_hermitian(oracle_lib):
    x = synth.uniform_bytes(12, 200, seed=9)
    v = oracle.correlate(x, full=True)
    np.testing.assert_array_equal(v[..., 0], v[..., 0].T)
    np.testing.assert_array_equal(v[..., 1], -v[..., 1].T)
    iu, ju = np.triu_indices(12)
    np.testing.assert_array_equal(v[iu, ju], oracle.correlate(x))


def test_additivity_in_time(oracle_lib):
    x = synth.uniform_bytes(20, 301, seed=10)
    for cut in (0, 1, 150, 300, 301):
        np.testing.assert_array_equal(oracle.correlate(x[:cut]) + oracle.correlate(x[cut:]),
                                      oracle.correlate(x))


def test_re_low_flag_reads_swapped_bytes(oracle_lib):
    x = synth.uniform_bytes(10, 64, seed=12)
    swapped = ((x << 4) | (x >> 4)).astype(np.uint8)
    np.testing.assert_array_equal(oracle.correlate(swapped, re_low=True), oracle.correlate(x))


def test_negated_imaginary_is_conjugate(oracle_lib):
    rng = _rng(13)
    re = rng.integers(-7, 8, size=(80, 9))
    im = rng.integers(-7, 8, size=(80, 9))
    a = oracle.correlate(synth.encode(re, im))
    b = oracle.correlate(synth.encode(re, -im))
    np.testing.assert_array_equal(b * np.array([1, -1]), a)


def test_phase_rotation_invariance(oracle_lib):
    # multiplying every input by j (a common phase) leaves V unchanged
    rng = _rng(14)
    re = rng.integers(-7, 8, size=(64, 11))
    im = rng.integers(-7, 8, size=(64, 11))
    np.testing.assert_array_equal(oracle.correlate(synth.encode(-im, re)),
                                  oracle.correlate(synth.encode(re, im)))


def test_flagged_inputs_zero_rows(oracle_lib):
    x = synth.chime_channel(40, 128, seed=15)
    idx = synth.flag_inputs(x, 5, seed=16)
    v = oracle.correlate(x, full=True)
    assert not v[idx].any() and not v[:, idx].any()


def test_row_stride_padding_ignored(oracle_lib):
    x = synth.uniform_bytes(13, 77, seed=17)
    padded = _rng(18).integers(0, 256, size=(77, 20), dtype=np.uint8)
    padded[:, :13] = x
    np.testing.assert_array_equal(oracle.correlate(padded, n_inputs=13), oracle.correlate(x))


def test_int32_bound_at_max_integration(oracle_lib):
    # The largest |term| per sample is 128 (both parts -8); 16,777,215 samples
    # of it reach 2,147,483,520 <= 2^31 - 1 and one more sample would not fit.
    worst = max(abs(_x(a) * _x(b).conjugate()).real for a in range(256) for b in range(256))
    re_max = max(abs((_x(a) * _x(b).conjugate()).real) for a in range(256) for b in range(256))
    im_max = max(abs((_x(a) * _x(b).conjugate()).imag) for a in range(256) for b in range(256))
    assert re_max == 128 and im_max == 120 and worst >= 128
    t_max = (2 ** 31 - 1) // 128
    assert t_max == 16_777_215
    assert 128 * t_max <= 2 ** 31 - 1 < 128 * (t_max + 1)


def test_empty_time_axis(oracle_lib):
    assert not oracle.correlate(np.zeros((0, 5), np.uint8)).any()


# ---------------------------------------------------------------------------
# Printed numbers from the paper
# ---------------------------------------------------------------------------

def test_eta_table_pins_triangle_count():
    """eta = dnu * N(N+1)/2 reproduces Table tab:corrs (autocorrelations
    included); N^2/2 and N(N-1)/2 do not."""
    rows = _read_rows("eta_table.txt")
    assert len(rows) == 13

    def ok(count, n, dnu, printed):
        digits = printed.split(".")[1] if "." in printed else ""
        half_unit = 0.5 * 10.0 ** (-len(digits))
        return abs(dnu * 1e6 * count(n) / 1e12 - float(printed)) <= half_unit + 1e-12

    consistent = [r for r in rows if r[4] == "1"]
    assert len(consistent) == 10
    for name, n, dnu, printed, _ in consistent:
        assert ok(oracle.tri, int(n), float(dnu), printed), name
    for wrong in (lambda n: n * n / 2, lambda n: n * (n - 1) / 2):
        assert not all(ok(wrong, int(n), float(d), p) for _, n, d, p, _ in consistent)


def test_data_rates_pin_formats():
    rates = {r[0]: float(r[1]) for r in _read_rows("data_rates.txt")}
    n, dnu = 2048, 400e6
    # 8 bits per complex sample (4 real + 4 imaginary)
    assert round(n * dnu * 8 / 1e12, 1) == rates["input_tbps"]
    # one 390 kHz channel (400 MHz / 1024) per GPU: 819.6 GcMAC/s, quoted as ~819
    assert abs(dnu / 1024 * oracle.tri(n) / 1e9 - rates["per_gpu_gcmac"]) < 1.0
    # 4 channels of 2048 inputs at 2.56 us per sample
    assert round(4 * n * (dnu / 1024) * 8 / 1e9, 1) == rates["samples_in_gbps_per_node"]
    # visibilities: N(N+1)/2 complex int32 (8 bytes) per channel, 4 channels, every 10 s
    assert round(4 * oracle.tri(n) * 8 * 8 / 10 / 1e9, 2) == rates["vis_out_gbps_per_node"]


# ---------------------------------------------------------------------------
# Planted mistakes: each mutated oracle must fail at least one pin
# ---------------------------------------------------------------------------

MUTANTS = {
    "offset_7": ("return (int)nib - 8;", "return (int)nib - 7;"),
    "nibble_order": ("re[i * T + t] = (int8_t)nibble_value(re_low ? lo : hi);",
                     "re[i * T + t] = (int8_t)nibble_value(re_low ? hi : lo);"),
    "re_sign": ("vr += (int64_t)ri[t] * rj[t] + (int64_t)ii[t] * ij[t];",
                "vr += (int64_t)ri[t] * rj[t] - (int64_t)ii[t] * ij[t];"),
    "dropped_term": ("vr += (int64_t)ri[t] * rj[t] + (int64_t)ii[t] * ij[t];",
                     "vr += (int64_t)ri[t] * rj[t];"),
    "conj_side": ("vi += (int64_t)ii[t] * rj[t] - (int64_t)ri[t] * ij[t];",
                  "vi += (int64_t)ri[t] * ij[t] - (int64_t)ii[t] * rj[t];"),
    "transposed_operand": ("const int8_t *rj = re + j * T, *ij = im + j * T;",
                           "const int8_t *rj = re + j * T, *ij = im + i * T;"),
    "dropped_sample": ("for (int64_t t = 0; t < T; ++t) {\n                /*",
                       "for (int64_t t = 1; t < T; ++t) {\n                /*"),
    "no_autos": ("for (int64_t j = (full ? 0 : i); j < N; ++j)",
                 "for (int64_t j = (full ? 0 : i + 1); j < N; ++j)"),
    "index": ("(i * N - i * (i - 1) / 2 + (j - i))", "(i * N - i * (i + 1) / 2 + (j - i))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name, oracle_lib):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(oracle._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        so = oracle.compile_source(path, os.path.join(d, "libmutant.so"))
        lib = oracle.load_library(so)
        failed = []
        for pin in PINS:
            try:
                pin(lambda s, **kw: oracle.correlate(s, _lib_override=lib, **kw))
            except AssertionError:
                failed.append(pin.__name__)
        assert failed, f"no pin catches mutant {name}"
