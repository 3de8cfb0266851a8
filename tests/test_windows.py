"""The sampled-window oracle helpers equal the whole-tensor oracle (CPU)."""
import numpy as np

from oracle import codec, nets
from synthetic import stand_in_weights, video_chunk
from tests import windows as wn


def test_windows_equal_whole_tensor_oracle():
    T, H, W, C = 4, 136, 200, 64
    fr = video_chunk(T, H, W, 3, seed=4)
    w = stand_in_weights(T, C)
    h, ww, _, _ = codec.latent_size(H, W)
    y = nets.analysis(fr, w)
    zu = nets.conv(y, w["h"], stride=2)
    zh = nets.rint_clamp(zu)
    mu, sig = nets.params(zh, w, h, ww)
    x = nets.synthesis(y, w, T, H, W)
    # corners, ragged right / bottom edges (W = 200 is not a multiple of 16), interior
    for r0, r1, c0, c1 in [(0, 4, 0, 4), (14, 18, 22, 26), (5, 9, 11, 15), (7, 13, 3, 6)]:
        np.testing.assert_allclose(wn.analysis_window(fr, w, h, ww, r0, r1, c0, c1),
                                   y[:, r0:r1, c0:c1], rtol=0, atol=1e-12)
        m, s = wn.params_window(zh, w, h, ww, r0, r1, c0, c1)
        np.testing.assert_allclose(m, mu[:, r0:r1, c0:c1], rtol=0, atol=1e-12)
        np.testing.assert_allclose(s, sig[:, r0:r1, c0:c1], rtol=0, atol=1e-12)
        xs = wn.synthesis_window(y, w, T, H, W, r0, r1, c0, c1)
        np.testing.assert_allclose(xs, x[:, :, 8 * r0:8 * r1, 8 * c0:8 * c1], rtol=0, atol=1e-12)
    for a0, a1, b0, b1 in [(0, 3, 0, 3), (6, 9, 10, 13), (2, 5, 4, 8)]:
        np.testing.assert_allclose(wn.hyper_window(y, w, a0, a1, b0, b1), zu[:, a0:a1, b0:b1],
                                   rtol=0, atol=1e-12)
