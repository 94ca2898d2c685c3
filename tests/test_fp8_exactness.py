"""The arithmetic the exact FP8 path rests on, checked on the CPU from the
OCP E4M3 format's definition (1 sign bit, 4 exponent bits with bias 7, 3
mantissa bits; exponent 0 is subnormal): every 4-bit sample value and its
negation has an exact code, every product of two such values is exact, and
the longest piece's fp32 sums stay below 2^24, where every integer is exact
and addition of integers is exact in any order."""
import numpy as np


def e4m3_value(code):
    s = -1.0 if code & 0x80 else 1.0
    e, m = (code >> 3) & 0xF, code & 7
    if e == 0:
        return s * (m / 8.0) * 2.0 ** (1 - 7)
    if e == 0xF and m == 7:
        return float("nan")
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def test_every_sample_value_and_its_negation_is_exact():
    values = {}                      # value -> its first code (+0 before -0)
    for c in range(256):
        if not np.isnan(e4m3_value(c)):
            values.setdefault(e4m3_value(c), c)
    for v in range(-8, 9):
        assert float(v) in values, v
    # the codes the kernel's tables hold, derived here from the definition
    assert [values[float(v)] for v in range(0, 9)] == [0x00, 0x38, 0x40, 0x44, 0x48, 0x4A, 0x4C, 0x4E, 0x50]
    assert all(values[float(-v)] == values[float(v)] | 0x80 for v in range(1, 9))


def test_products_and_piece_sums_are_exact():
    prods = {a * b for a in range(-8, 9) for b in range(-8, 9)}
    assert max(abs(p) for p in prods) == 64
    assert all(np.float32(p) == p for p in prods)
    # Re per sample: R_i R_j + I_i I_j <= 128; the longest FP8 piece
    max_stages = ((1 << 17) - 1) // 64
    assert max_stages == 2047
    assert 128 * 64 * max_stages < 2 ** 24
    # every integer below 2^24 survives fp32, 2^24 + 1 does not
    assert float(np.float32(2 ** 24 - 1)) == 2 ** 24 - 1
    assert float(np.float32(2 ** 24 + 1)) != 2 ** 24 + 1
