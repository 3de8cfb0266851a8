"""Pins for the scale table, index, symbols and CDF tables (Sec. 3.4 readings)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import entropy


def test_scales_closed_form():
    s = entropy.scales()
    assert s[0] == pytest.approx(0.11, rel=1e-15)
    assert s[63] == pytest.approx(64.0, rel=1e-14)
    ratio = (64 / 0.11) ** (1 / 63)
    np.testing.assert_allclose(s[1:] / s[:-1], ratio, rtol=1e-13)
    assert ratio == pytest.approx(1.10633, abs=1e-5)


def test_thresholds_are_geometric_midpoints():
    s = entropy.scales()
    t = entropy.thresholds()
    assert t.dtype == np.float32 and t.shape == (63,)
    for j in range(63):
        assert s[j] < t[j] < s[j + 1]
        assert abs(float(t[j]) - math.sqrt(s[j] * s[j + 1])) <= 1e-7 * float(t[j])


def test_index_special_cases():
    s = entropy.scales()
    t = entropy.thresholds().astype(np.float64)
    assert entropy.scale_index(np.array(0.11)) == 0
    assert entropy.scale_index(np.array(64.0)) == 63
    np.testing.assert_array_equal(entropy.scale_index(s), np.arange(64))
    # a value exactly on a threshold goes up; the float32 just below stays down
    below = np.nextafter(entropy.thresholds(), np.float32(0)).astype(np.float64)
    np.testing.assert_array_equal(entropy.scale_index(t), np.arange(1, 64))
    np.testing.assert_array_equal(entropy.scale_index(below), np.arange(0, 63))
    grid = np.exp(np.linspace(math.log(0.11), math.log(64), 20001))
    assert np.all(np.diff(entropy.scale_index(grid).astype(int)) >= 0)
    # nearest in the log domain
    k = entropy.scale_index(grid).astype(int)
    d_sel = np.abs(np.log(grid) - np.log(s[k]))
    d_all = np.abs(np.log(grid)[:, None] - np.log(s)[None, :]).min(axis=1)
    assert np.all(d_sel <= d_all + 1e-6)


def test_symbolise_special_cases():
    y = np.array([0.5, -0.5, 1.5, 2.5, 100.0, -100.0, 0.49, 3.0])
    mu = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0])
    np.testing.assert_array_equal(entropy.symbolise(y, mu), np.array([0, 0, 2, 2, 32, -32, 0, 2]) + 32)


def _scipy_pmf(s):
    r = np.arange(-32, 33)
    hi = norm.cdf((r + 0.5) / s)
    lo = norm.cdf((r - 0.5) / s)
    lo[0] = 0.0
    hi[-1] = 1.0
    return hi - lo


def test_pmf_matches_scipy():
    for s in entropy.scales():
        np.testing.assert_allclose(entropy.gaussian_pmf(float(s)), _scipy_pmf(float(s)),
                                   rtol=1e-9, atol=1e-15)
        assert entropy.gaussian_pmf(float(s)).sum() == pytest.approx(1.0, abs=1e-12)


def test_cdf_table_invariants():
    freq, cum = entropy.cdf_tables()
    M = entropy.M
    assert freq.shape == (64, 65) and cum.shape == (64, 65)
    assert np.all(freq.sum(axis=1) == M)
    assert np.all(freq >= 1)
    assert np.all(freq == freq[:, ::-1])
    assert np.all(np.diff(cum, axis=1) > 0) and np.all(cum[:, 0] == 0)
    assert np.all(cum[:, -1] + freq[:, -1] == M)
    assert np.all(np.diff(freq[:, 32]) <= 0)
    assert freq.max() < 65536 and cum.max() < 65536
    for k, s in enumerate(entropy.scales()):
        p = _scipy_pmf(float(s))
        assert np.all(np.abs(freq[k] - M * p) <= 66)


def test_cdf_table_hand_values():
    freq, _ = entropy.cdf_tables()
    # sigma = 0.11: the centre holds all but the 64 minimum counts
    assert freq[0, 32] == 65536 - 64
    # sigma = 64: nearly uniform; the edges absorb the tails
    p = _scipy_pmf(64.0)
    assert freq[63, 0] == 1 + math.floor(p[0] * (65536 - 65))
    assert freq[63, 1] == 1 + math.floor(p[1] * (65536 - 65))


def test_ideal_bits():
    freq = np.array([[1 << 15, 1 << 15], [1 << 14, 3 << 14]])
    assert entropy.ideal_bits([0, 1, 1], [0, 0, 1], freq) == pytest.approx(1 + 1 + (16 - math.log2(3 << 14)))
