"""Pins for the colour conversions around the YUV444 interface (supplementary
RGB section; BT.709 full range): closed-form primaries and greys, luma weights,
exact round trips, and the 4:2:0 resampling identities."""
import numpy as np
import pytest

from oracle import color


def px(r, g, b):
    return np.array([r, g, b], np.float64).reshape(3, 1, 1)


def test_greys_have_centred_chroma():
    for v in (0.0, 0.25, 0.5, 1.0):
        y, cb, cr = color.rgb_to_yuv444(px(v, v, v)).ravel()
        assert abs(y - v) < 1e-15 and abs(cb - 0.5) < 1e-15 and abs(cr - 0.5) < 1e-15


def test_primaries_closed_form():
    # BT.709: red has luma Kr and Cr at the top of the range, blue likewise Cb
    y, cb, cr = color.rgb_to_yuv444(px(1, 0, 0)).ravel()
    assert abs(y - 0.2126) < 1e-15 and abs(cr - 1.0) < 1e-15
    assert abs(cb - (0.5 - 0.2126 / (2 * (1 - 0.0722)))) < 1e-15
    y, cb, cr = color.rgb_to_yuv444(px(0, 0, 1)).ravel()
    assert abs(y - 0.0722) < 1e-15 and abs(cb - 1.0) < 1e-15
    y, cb, cr = color.rgb_to_yuv444(px(0, 1, 0)).ravel()
    assert abs(y - 0.7152) < 1e-15
    assert color.KR + color.KG + color.KB == pytest.approx(1.0, abs=1e-15)


def test_round_trip_is_identity():
    rng = np.random.default_rng(1)
    rgb = rng.random((2, 3, 6, 10))
    back = color.yuv444_to_rgb(color.rgb_to_yuv444(rgb), clamp=False)
    np.testing.assert_allclose(back, rgb, rtol=0, atol=1e-14)
    # every RGB in [0, 1] maps to Y, Cb, Cr in [0, 1]
    yuv = color.rgb_to_yuv444(rng.random((1, 3, 64, 64)))
    assert yuv.min() >= -1e-15 and yuv.max() <= 1 + 1e-15


def test_output_clamp():
    # a YUV triple outside the RGB cube converts and clamps into [0, 1]
    out = color.yuv444_to_rgb(np.array([1.0, 1.0, 1.0]).reshape(3, 1, 1))
    assert out.min() >= 0.0 and out.max() <= 1.0


def test_420_resampling_identities():
    rng = np.random.default_rng(2)
    T, H, W = 2, 8, 12
    y = rng.random((T, H, W))
    cb = rng.random((T, H // 2, W // 2))
    cr = rng.random((T, H // 2, W // 2))
    full = color.yuv420_to_444(y, cb, cr)
    assert full.shape == (T, 3, H, W)
    y2, cb2, cr2 = color.yuv444_to_420(full)
    np.testing.assert_array_equal(y2, y)
    np.testing.assert_allclose(cb2, cb, atol=1e-15)
    np.testing.assert_allclose(cr2, cr, atol=1e-15)
    # the chroma mean is preserved by the block average
    x = rng.random((T, 3, H, W))
    _, cbd, crd = color.yuv444_to_420(x)
    assert abs(cbd.mean() - x[:, 1].mean()) < 1e-14 and abs(crd.mean() - x[:, 2].mean()) < 1e-14
    # brute force on one block
    assert abs(cbd[1, 2, 3] - x[1, 1, 4:6, 6:8].mean()) < 1e-15
    with pytest.raises(ValueError):
        color.yuv444_to_420(rng.random((1, 3, 5, 4)))
