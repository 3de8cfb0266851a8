"""The entropy-parameter conv (Sec. 3.4: a 3x3 conv over the nearest x2
upsampling of z_hat) written as four 2x2 convs over z_hat, one per output
parity class, with summed weights: the form the library's kernel computes.

Pinned against the oracle's own up2 + conv in float64 on even latent sizes
(the codec's latent is always even: frames are padded to multiples of 16 and
the latent is 1/8 of that), including zero padding at every border, and
shown to fail for an odd (cropped) size, which the library rejects."""
import numpy as np
import pytest

from oracle import nets

# kernel rows gathered by hyper-latent row offset r (0, 1) for output parity p
ROWS = {0: ((0,), (1, 2)), 1: ((0, 1), (2,))}


def merged_weights(w):
    """[4 classes][4 taps][cout][cin] from OIHW 3x3 weights (float64)."""
    out = np.zeros((4, 4) + w.shape[:2])
    for cls in range(4):
        py, px = divmod(cls, 2)
        for t in range(4):
            r, q = divmod(t, 2)
            for dy in ROWS[py][r]:
                for dx in ROWS[px][q]:
                    out[cls, t] += w[:, :, dy, dx]
    return out


def params_by_class(z, w, h, ww):
    """Output (2qy + py, 2qx + px) = sum over r, q of Wm[cls, 2r + q] .
    z[qy - 1 + py + r, qx - 1 + px + q] (zero outside z)."""
    cz, hz, wz = z.shape
    wm = merged_weights(w)
    zp = np.pad(z, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], h, ww))
    for cls in range(4):
        py, px = divmod(cls, 2)
        acc = np.zeros((w.shape[0], hz, wz))
        for t in range(4):
            r, q = divmod(t, 2)
            win = zp[:, py + r:py + r + hz, px + q:px + q + wz]
            acc += np.einsum("oc,chw->ohw", wm[cls, t], win)
        out[:, py::2, px::2] = acc[:, :(h - py + 1) // 2, :(ww - px + 1) // 2]
    return out


@pytest.mark.parametrize("hz,wz", [(1, 1), (2, 3), (5, 4), (7, 9)])
def test_four_classes_equal_the_upsampled_conv(hz, wz):
    rng = np.random.default_rng(hz * 31 + wz)
    cz, cout = 6, 10
    z = rng.integers(-32, 33, size=(cz, hz, wz)).astype(np.float64)
    w = rng.standard_normal((cout, cz, 3, 3))
    h, ww = 2 * hz, 2 * wz
    ref = nets.conv(nets.up2(z, h, ww), w)
    np.testing.assert_allclose(params_by_class(z, w, h, ww), ref, rtol=1e-12, atol=1e-11)


def test_merged_weights_sum_every_tap_once_per_class():
    w = np.random.default_rng(3).standard_normal((4, 5, 3, 3))
    wm = merged_weights(w)
    for cls in range(4):
        np.testing.assert_allclose(wm[cls].sum(axis=0), w.sum(axis=(2, 3)), rtol=1e-12, atol=1e-12)


def test_odd_latent_is_not_that_form():
    """A cropped upsampling (odd latent height) breaks the merge on the last
    row: the library accepts even latents only."""
    rng = np.random.default_rng(5)
    z = rng.integers(-32, 33, size=(3, 3, 3)).astype(np.float64)
    w = rng.standard_normal((4, 3, 3, 3))
    h, ww = 5, 6
    ref = nets.conv(nets.up2(z, h, ww), w)
    got = params_by_class(z, w, h, ww)
    assert not np.allclose(got[:, -1], ref[:, -1])
    np.testing.assert_allclose(got[:, :-1], ref[:, :-1], rtol=1e-12, atol=1e-11)
