"""Pins of the FP8 numerics model used by the GPU FP8 tests (OCP E4M3 and
bfloat16 rounding, values fixed by the formats' definitions)."""
import numpy as np

from tests import fp8_model as m


def test_e4m3_values():
    cases = {
        0.0: 0.0, 448.0: 448.0, 500.0: 448.0, -1e9: -448.0,   # saturation
        1.0: 1.0, 1.0625: 1.0,            # tie between m=0 and m=1 -> even
        1.1875: 1.25,                     # tie between m=1 and m=2 -> even
        232.0: 224.0, 248.0: 256.0,       # ties at the top binades
        2.0 ** -6: 2.0 ** -6,             # smallest normal
        2.0 ** -9: 2.0 ** -9,             # smallest subnormal
        2.0 ** -10: 0.0,                  # half the smallest subnormal -> even (0)
        3 * 2.0 ** -10: 2.0 ** -8,        # 1.5 steps -> 2 steps
        7 * 2.0 ** -9: 7 * 2.0 ** -9,     # largest subnormal
        -0.3: -0.3125,
    }
    for x, want in cases.items():
        assert m.e4m3(x) == want, (x, m.e4m3(x), want)


def test_e4m3_grid_is_the_256_code_table():
    # every value of the grid maps to itself; midpoints go to the even code
    vals = []
    for e in range(16):
        for q in range(8):
            if e == 15 and q == 7:
                continue                      # NaN code
            vals.append(q * 2.0 ** -9 if e == 0 else (1 + q / 8) * 2.0 ** (e - 7))
    vals = np.array(vals)
    assert vals.max() == 448.0 and len(vals) == 127
    np.testing.assert_array_equal(m.e4m3(vals), vals)
    mids = (vals[1:] + vals[:-1]) / 2
    got = m.e4m3(mids)
    codes = np.searchsorted(vals, got)
    assert np.all(codes % 2 == 0)             # even mantissa wins every tie
    assert np.all((got == vals[:-1]) | (got == vals[1:]))


def test_bf16_rounding():
    assert m.bf16(1.0) == 1.0
    assert m.bf16(1 + 2.0 ** -8) == 1.0                   # tie -> even
    assert m.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6     # tie -> even (up)
    assert m.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    x = np.random.default_rng(0).standard_normal(1000)
    r = m.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
