"""Oracle values at sampled latent windows of full-size chunks (tests only).

A full 1080p chunk is too large for the float64 oracle to run whole inside a
test, but every output depends only on a bounded neighbourhood: each 3x3 conv
widens the receptive field by one latent position, so a window grown by the
number of convs on every side (clipped at the true borders, where the conv's
zero padding is the real one) gives exact values in its centre.  The
functions below run the oracle's own steps (pad16, patchify, conv, up2,
pixel shuffle) on such grown windows.
"""
import numpy as np

from oracle import entropy, nets


def _grow(r0, r1, n, m):
    return max(0, r0 - m), min(n, r1 + m)


def analysis_window(frames, wts, h, w, r0, r1, c0, c1):
    """y (C, r1-r0, c1-c0) at latent rows [r0, r1), cols [c0, c1)."""
    T, _, H, W = frames.shape
    e0, e1 = _grow(r0, r1, h, 3)
    f0, f1 = _grow(c0, c1, w, 3)
    rows = np.minimum(np.arange(8 * e0, 8 * e1), H - 1)     # pad16 edge replication
    cols = np.minimum(np.arange(8 * f0, 8 * f1), W - 1)
    X = nets.patchify(frames[:, :, rows][:, :, :, cols].astype(np.float64))
    a = nets.relu(nets.conv(X, wts["a1"]))
    a = nets.relu(nets.conv(a, wts["a2"]))
    y = nets.conv(a, wts["a3"])
    return y[:, r0 - e0:r1 - e0, c0 - f0:c1 - f0]


def hyper_window(y_chw, wts, zr0, zr1, zc0, zc1):
    """Unrounded z (32, ...) at hyper rows [zr0, zr1), cols [zc0, zc1) from a
    full latent y (C, h, w)."""
    _, h, w = y_chw.shape
    e0, e1 = max(0, 2 * zr0 - 1), min(h, 2 * zr1 + 1)
    f0, f1 = max(0, 2 * zc0 - 1), min(w, 2 * zc1 + 1)
    sub = y_chw[:, e0:e1, f0:f1]
    # a stride-2 conv on the sub-window: output (a, b) reads rows 2a-1..2a+1
    # of the full tensor; shift so the sub-window's row 0 is full row e0
    pad = np.zeros((sub.shape[0], (e1 - e0) + 2, (f1 - f0) + 2))
    oy, ox = e0 - (2 * zr0 - 1), f0 - (2 * zc0 - 1)
    pad[:, oy:oy + e1 - e0, ox:ox + f1 - f0] = sub
    out = np.zeros((wts["h"].shape[0], zr1 - zr0, zc1 - zc0))
    for ky in range(3):
        for kx in range(3):
            patch = pad[:, ky:ky + 2 * (zr1 - zr0 - 1) + 1:2, kx:kx + 2 * (zc1 - zc0 - 1) + 1:2]
            out += np.tensordot(wts["h"][:, :, ky, kx].astype(np.float64), patch, axes=(1, 0))
    return out


def params_window(zhat_chw, wts, h, w, r0, r1, c0, c1):
    """(mu, sigma) at latent rows [r0, r1), cols [c0, c1) from a full z_hat."""
    e0, e1 = _grow(r0, r1, h, 1)
    f0, f1 = _grow(c0, c1, w, 1)
    up = nets.up2(zhat_chw.astype(np.float64), h, w)[:, e0:e1, f0:f1]
    C = wts["p"].shape[0] // 2
    P = nets.conv(up, wts["p"])[:, r0 - e0:r1 - e0, c0 - f0:c1 - f0]
    sigma = np.clip(nets.softplus(P[C:]), entropy.SIGMA_MIN, entropy.SIGMA_MAX)
    return P[:C], sigma


def synthesis_window(yhat_chw, wts, T, H, W, r0, r1, c0, c1):
    """Frames (T, 3, rows, cols) of the pixels of latent rows [r0, r1), cols
    [c0, c1), cropped to the frame, from a full y_hat (C, h, w)."""
    _, h, w = yhat_chw.shape
    e0, e1 = _grow(r0, r1, h, 6)
    f0, f1 = _grow(c0, c1, w, 6)
    F = nets.chunk_decoder(yhat_chw[:, e0:e1, f0:f1].astype(np.float64), wts)
    out = []
    for t in range(T):
        g = nets.relu(nets.conv(F, wts[f"k1_{t}"]))
        g = nets.relu(nets.conv(g, wts[f"k2_{t}"]))
        o = nets.conv(g, wts[f"k3_{t}"])[:, r0 - e0:r1 - e0, c0 - f0:c1 - f0]
        px = nets.pixel_shuffle8(o)
        out.append(np.clip(px[:, :max(0, min(8 * r1, H) - 8 * r0), :max(0, min(8 * c1, W) - 8 * c0)],
                           0.0, 1.0))
    return np.stack(out)
