"""Frame colour formats around the codec's YUV444 interface.

Test infrastructure only (see the package docstring).

The supplementary material's RGB section: the codec takes and returns YUV444
as its one interface; RGB and YUV420 video are converted to YUV444 before
inference and back afterwards, RGB with BT.709 (chosen over BT.601 for its
rate at similar quality).  Readings where the text gives no detail:

  * full range, all values in [0, 1]; chroma centred at 1/2;
  * BT.709 luma weights Kr = 0.2126, Kb = 0.0722, Kg = 1 - Kr - Kb:
        Y  = Kr R + Kg G + Kb B
        Cb = (B - Y) / (2 (1 - Kb)) + 1/2
        Cr = (R - Y) / (2 (1 - Kr)) + 1/2
    and its exact inverse;
  * YUV420 is planar (Y at H x W, Cb and Cr at H/2 x W/2, H and W even);
    4:2:0 -> 4:4:4 repeats each chroma sample over its 2 x 2 block, and
    4:4:4 -> 4:2:0 takes the mean of the block;
  * on output the codec's YUV444 (already clamped to [0, 1]) is converted
    and clamped to [0, 1] again.

Frames are (T, 3, H, W) arrays of planes; a YUV420 chunk is the tuple
(Y (T, H, W), Cb (T, H/2, W/2), Cr (T, H/2, W/2)).

Pins: primaries and grey levels against the closed forms, the luma weights
summing to one, the round trip RGB -> YUV -> RGB, and the 4:2:0 identities
(down(up(c)) = c; up(down(x)) = x for 2 x 2-constant chroma; the mean is
preserved).
"""
from __future__ import annotations

import numpy as np

KR = 0.2126
KB = 0.0722
KG = 1.0 - KR - KB


def rgb_to_yuv444(rgb: np.ndarray) -> np.ndarray:
    """BT.709 full range, (..., 3, H, W) RGB planes -> Y, Cb, Cr planes."""
    x = np.asarray(rgb, dtype=np.float64)
    r, g, b = x[..., 0, :, :], x[..., 1, :, :], x[..., 2, :, :]
    y = KR * r + KG * g + KB * b
    cb = (b - y) / (2.0 * (1.0 - KB)) + 0.5
    cr = (r - y) / (2.0 * (1.0 - KR)) + 0.5
    return np.stack([y, cb, cr], axis=-3)


def yuv444_to_rgb(yuv: np.ndarray, clamp: bool = True) -> np.ndarray:
    """Inverse of rgb_to_yuv444, then (by default) clamped to [0, 1]."""
    x = np.asarray(yuv, dtype=np.float64)
    y, cb, cr = x[..., 0, :, :], x[..., 1, :, :], x[..., 2, :, :]
    r = y + 2.0 * (1.0 - KR) * (cr - 0.5)
    b = y + 2.0 * (1.0 - KB) * (cb - 0.5)
    g = (y - KR * r - KB * b) / KG
    out = np.stack([r, g, b], axis=-3)
    return np.clip(out, 0.0, 1.0) if clamp else out


def yuv420_to_444(y: np.ndarray, cb: np.ndarray, cr: np.ndarray) -> np.ndarray:
    """(T, H, W), (T, H/2, W/2) x 2 -> (T, 3, H, W): chroma repeated over 2 x 2."""
    up = lambda c: np.repeat(np.repeat(np.asarray(c, np.float64), 2, axis=-2), 2, axis=-1)  # noqa: E731
    return np.stack([np.asarray(y, np.float64), up(cb), up(cr)], axis=-3)


def yuv444_to_420(yuv: np.ndarray):
    """(T, 3, H, W) -> (Y, Cb, Cr) with chroma the mean of each 2 x 2 block."""
    x = np.asarray(yuv, dtype=np.float64)
    T, _, H, W = x.shape
    if H % 2 or W % 2:
        raise ValueError("4:2:0 needs even H and W")
    down = lambda c: c.reshape(T, H // 2, 2, W // 2, 2).mean(axis=(2, 4))  # noqa: E731
    return x[:, 0], down(x[:, 1]), down(x[:, 2])
