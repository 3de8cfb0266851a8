"""Pins for the DC block (supplementary material, DC-block section; structure
read as depth-wise 3x3 between point-wise mixings plus a point-wise
feed-forward stage, each with a residual connection): brute-force sums,
torch's grouped conv2d, the full-conv special case, and the residual
identities."""
import itertools

import numpy as np
import torch
import torch.nn.functional as F

from oracle import dcblock, nets
from synthetic import dc_block_weights, feature_map


def test_pointwise_bruteforce():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 3, 4))
    w = rng.standard_normal((7, 5)).astype(np.float32)
    out = dcblock.pointwise(x, w)
    for o, v, u in itertools.product(range(7), range(3), range(4)):
        want = sum(float(w[o, i]) * x[i, v, u] for i in range(5))
        assert abs(out[o, v, u] - want) < 1e-12


def test_depthwise_matches_torch_and_diagonal_conv():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 5, 9))
    w = rng.standard_normal((6, 3, 3)).astype(np.float32)
    out = dcblock.depthwise3x3(x, w)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w.astype(np.float64))[:, None],
                   padding=1, groups=6)[0].numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    full = np.zeros((6, 6, 3, 3), np.float32)
    for c in range(6):
        full[c, c] = w[c]
    np.testing.assert_allclose(out, nets.conv(x, full), rtol=1e-12, atol=1e-12)


def test_block_against_torch_composition():
    C, h, w = 16, 6, 10
    x = feature_map(C, h, w, seed=1).astype(np.float64)
    wt = dc_block_weights(C, seed=3)
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))  # noqa: E731
    X = t(x)[None]
    T = F.relu(F.conv2d(X, t(wt["pw1"])[:, :, None, None]))
    D = F.conv2d(T, t(wt["dw"])[:, None], padding=1, groups=C)
    X1 = X + F.conv2d(D, t(wt["pw2"])[:, :, None, None])
    U = F.relu(F.conv2d(X1, t(wt["pw3"])[:, :, None, None]))
    Y = X1 + F.conv2d(U, t(wt["pw4"])[:, :, None, None])
    np.testing.assert_allclose(dcblock.dc_block(x, wt), Y[0].numpy(), rtol=1e-12, atol=1e-12)


def test_residual_identities():
    C, h, w = 8, 4, 4
    x = feature_map(C, h, w, seed=2).astype(np.float64)
    wt = dc_block_weights(C, seed=4)
    z = dict(wt, pw2=np.zeros_like(wt["pw2"]), pw4=np.zeros_like(wt["pw4"]))
    np.testing.assert_array_equal(dcblock.dc_block(x, z), x)
    # with pw4 zero the block is x + pw2 dw relu(pw1 x)
    z4 = dict(wt, pw4=np.zeros_like(wt["pw4"]))
    want = x + dcblock.pointwise(dcblock.depthwise3x3(np.maximum(dcblock.pointwise(x, wt["pw1"]), 0),
                                                      wt["dw"]), wt["pw2"])
    np.testing.assert_allclose(dcblock.dc_block(x, z4), want, rtol=1e-12, atol=1e-12)


def test_weight_recipe_shapes():
    wt = dc_block_weights(128)
    assert wt["pw1"].shape == (128, 128) and wt["dw"].shape == (128, 3, 3)
    assert wt["pw3"].shape == (256, 128) and wt["pw4"].shape == (128, 256)
    assert all(v.dtype == np.float32 for v in wt.values())
