"""Pins for the oracle's transforms (Sec. 3.1-3.2 stand-in) against brute force
and independent library routines."""
import itertools
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import nets
from synthetic import stand_in_weights, video_chunk


def brute_conv(x, wt, stride):
    cin, H, W = x.shape
    cout = wt.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    out = np.zeros((cout, Ho, Wo))
    for o, v, u, i, ky, kx in itertools.product(range(cout), range(Ho), range(Wo), range(cin),
                                                range(3), range(3)):
        yy, xx = stride * v + ky - 1, stride * u + kx - 1
        if 0 <= yy < H and 0 <= xx < W:
            out[o, v, u] += float(wt[o, i, ky, kx]) * float(x[i, yy, xx])
    return out


@pytest.mark.parametrize("shape,stride", [((2, 5, 7), 1), ((2, 5, 7), 2), ((3, 4, 6), 2),
                                          ((1, 1, 1), 1), ((2, 3, 2), 2)])
def test_conv_bruteforce(shape, stride):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(shape)
    wt = rng.standard_normal((3, shape[0], 3, 3)).astype(np.float32)
    np.testing.assert_allclose(nets.conv(x, wt, stride), brute_conv(x, wt, stride),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_torch(stride):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((6, 11, 9))
    wt = rng.standard_normal((5, 6, 3, 3)).astype(np.float32)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(wt.astype(np.float64)),
                   stride=stride, padding=1)[0].numpy()
    np.testing.assert_allclose(nets.conv(x, wt, stride), ref, rtol=1e-12, atol=1e-12)


def test_conv_kernel_orientation():
    # A single tap at (ky, kx) = (0, 2) moves content by (+1, -1): out[v, u] = x[v-1, u+1].
    x = np.arange(20, dtype=np.float64).reshape(1, 4, 5)
    wt = np.zeros((1, 1, 3, 3), np.float32)
    wt[0, 0, 0, 2] = 1.0
    out = nets.conv(x, wt)
    assert out[0, 2, 1] == x[0, 1, 2]
    assert out[0, 0, 0] == 0.0 and out[0, 3, 4] == 0.0


def test_pad16_matches_replicate():
    fr = np.random.default_rng(5).random((2, 3, 20, 35))
    ref = F.pad(torch.from_numpy(fr), (0, 48 - 35, 0, 32 - 20), mode="replicate").numpy()
    np.testing.assert_array_equal(nets.pad16(fr), ref)
    assert nets.padded_size(1080, 1920) == (1088, 1920)
    assert nets.padded_size(480, 832) == (480, 832)
    assert nets.padded_size(2160, 3840) == (2160, 3840)


def test_patchify_matches_pixel_unshuffle():
    fr = np.random.default_rng(6).random((3, 3, 16, 32))
    ref = torch.cat([F.pixel_unshuffle(torch.from_numpy(fr[t])[None], 8)[0] for t in range(3)])
    X = nets.patchify(fr)
    np.testing.assert_array_equal(X, ref.numpy())
    # the explicit index formula
    t, c, i, j, v, u = 2, 1, 3, 5, 1, 2
    assert X[t * 192 + c * 64 + i * 8 + j, v, u] == fr[t, c, 8 * v + i, 8 * u + j]


def test_pixel_shuffle_matches_torch_and_inverts():
    o = np.random.default_rng(7).standard_normal((192, 3, 5))
    ref = F.pixel_shuffle(torch.from_numpy(o)[None], 8)[0].numpy()
    np.testing.assert_array_equal(nets.pixel_shuffle8(o), ref)
    fr = np.random.default_rng(8).random((1, 3, 24, 40))
    np.testing.assert_array_equal(nets.pixel_shuffle8(nets.patchify(fr)), fr[0])


def test_up2_matches_nearest():
    z = np.random.default_rng(9).standard_normal((4, 3, 5))
    ref = F.interpolate(torch.from_numpy(z)[None], scale_factor=2, mode="nearest")[0].numpy()
    np.testing.assert_array_equal(nets.up2(z, 6, 10), ref)
    np.testing.assert_array_equal(nets.up2(z, 5, 9), ref[:, :5, :9])


def test_softplus():
    assert nets.softplus(np.array(0.0)) == pytest.approx(math.log(2.0), abs=1e-15)
    assert nets.softplus(np.array(40.0)) == 40.0 + math.log1p(math.exp(-40.0))
    assert nets.softplus(np.array(-30.0)) == pytest.approx(math.exp(-30.0), rel=1e-12)
    x = np.linspace(-25, 25, 1001)
    ref = F.softplus(torch.from_numpy(x), beta=1, threshold=1000).numpy()
    np.testing.assert_allclose(nets.softplus(x), ref, rtol=1e-14, atol=1e-300)


def test_rint_clamp():
    x = np.array([0.5, -0.5, 1.5, -1.5, 2.5, 2.4999, 40.0, -40.0, 31.5, -32.5])
    np.testing.assert_array_equal(nets.rint_clamp(x), [0, 0, 2, -2, 2, 2, 32, -32, 32, -32])


def _torch_analysis(fr, w):
    T, _, H, W = fr.shape
    Hp, Wp = nets.padded_size(H, W)
    x = F.pad(torch.from_numpy(fr.astype(np.float64)), (0, Wp - W, 0, Hp - H), mode="replicate")
    X = torch.cat([F.pixel_unshuffle(x[t:t + 1], 8) for t in range(T)], dim=1)
    tw = {k: torch.from_numpy(v.astype(np.float64)) for k, v in w.items()}
    a = F.relu(F.conv2d(X, tw["a1"], padding=1))
    a = F.relu(F.conv2d(a, tw["a2"], padding=1))
    return F.conv2d(a, tw["a3"], padding=1)[0].numpy(), tw


def test_analysis_and_params_compose_like_torch():
    T, H, W, C = 2, 24, 40, 8
    fr = video_chunk(T, H, W, 2, seed=11)
    w = stand_in_weights(T, C)
    w["p"] = w["p"][: 2 * C]
    y = nets.analysis(fr, w)
    ref, tw = _torch_analysis(fr, w)
    np.testing.assert_allclose(y, ref, rtol=1e-10, atol=1e-10)
    zh = nets.hyper(y, w)
    zt = torch.round(F.conv2d(torch.from_numpy(y)[None], tw["h"], stride=2, padding=1))
    np.testing.assert_array_equal(zh, torch.clamp(zt, -32, 32)[0].numpy())
    h, ww = y.shape[1:]
    mu, sigma = nets.params(zh, w, h, ww)
    U = F.interpolate(torch.from_numpy(zh)[None], scale_factor=2, mode="nearest")[:, :, :h, :ww]
    P = F.conv2d(U, tw["p"], padding=1)[0]
    np.testing.assert_allclose(mu, P[:C].numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sigma, torch.clamp(F.softplus(P[C:], threshold=1000), 0.11, 64).numpy(),
                               rtol=1e-12, atol=1e-12)


def test_synthesis_composes_like_torch():
    T, H, W, C = 2, 20, 36, 8
    w = stand_in_weights(T, C)
    Hp, Wp = nets.padded_size(H, W)
    yh = np.random.default_rng(12).standard_normal((C, Hp // 8, Wp // 8))
    out = nets.synthesis(yh, w, T, H, W)
    tw = {k: torch.from_numpy(v.astype(np.float64)) for k, v in w.items()}
    f = torch.from_numpy(yh)[None]
    for k in ("d1", "d2", "d3"):
        f = F.relu(F.conv2d(f, tw[k], padding=1))
    for t in range(T):
        g = F.relu(F.conv2d(f, tw[f"k1_{t}"], padding=1))
        g = F.relu(F.conv2d(g, tw[f"k2_{t}"], padding=1))
        o = F.pixel_shuffle(F.conv2d(g, tw[f"k3_{t}"], padding=1), 8)[0, :, :H, :W]
        np.testing.assert_allclose(out[t], torch.clamp(o, 0, 1).numpy(), rtol=1e-10, atol=1e-10)


def test_generator_is_seeded_and_shaped():
    a = video_chunk(4, 64, 64, 3, seed=1)
    b = video_chunk(4, 64, 64, 3, seed=1)
    c = video_chunk(4, 64, 64, 3, seed=2)
    assert a.shape == (4, 3, 64, 64) and a.dtype == np.float32
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() <= 1.0
    w = stand_in_weights(4, 64)
    assert w["a1"].shape == (64, 768, 3, 3) and w["k3_3"].shape == (192, 64, 3, 3)
    assert abs(float(w["a2"].std()) - math.sqrt(2 / (64 * 9))) < 0.01
