"""Numerics model of the FP8 synthesis path, for tests only.

It applies, in float64, exactly the roundings the mixed-precision decoder
declares: the latent and d1's weights in bfloat16, every stored activation
rounded to bfloat16 after ReLU, the layers after d1 on FP8 E4M3 (OCP: bias 7,
largest finite 448, round to nearest even, saturating) operands with one
per-tensor activation scale amax / 448 (amax of the stored producer output,
taken over all frame heads together for the stacked head layers) and one
weight scale amax / 448 per output channel.  Only accumulation order and
float32 accumulation separate it from the GPU, so the two agree closely; the
error of the path itself is measured against the FP64 oracle separately.

The convolutions are the oracle's direct sums; the roundings are written
here from the formats' definitions and share nothing with the library.
"""
import numpy as np

from oracle import nets


def bf16(x):
    """Round float64 values to bfloat16 (nearest even) via float32."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3(x):
    """Round to the nearest OCP E4M3 value (ties to even), saturating at 448."""
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), 448.0)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)          # below 2^-6 the spacing stays 2^-9
    step = np.exp2(e - 3.0)
    q = np.rint(a / step) * step     # rint rounds half to even
    return np.sign(x) * np.minimum(q, 448.0)


def _wq(w):
    """Per-output-channel E4M3 weights and their scales."""
    amax = np.abs(w).reshape(w.shape[0], -1).max(axis=1)
    s = np.where(amax > 0, (amax.astype(np.float32) / np.float32(448.0)).astype(np.float64), 1.0)
    return e4m3(w / s[:, None, None, None]), s


def fp8_conv(x, amax, w, with_bound=False):
    """conv(x, w) on E4M3 operands, rescaled (no activation applied); x is
    (Cin, h, w), amax the scale source of x.  with_bound also returns the
    rescaled sum of |products|, which bounds float32 accumulation error."""
    qs = amax / 448.0 if amax > 0 else 1.0
    qinv = np.float32(448.0) / np.float32(amax) if amax > 0 else np.float32(1.0)
    xq = e4m3(np.minimum((x.astype(np.float32) * qinv).astype(np.float64), 448.0))
    wq, ws = _wq(w)
    sc = (np.float32(qs) * ws.astype(np.float32)).astype(np.float64)[:, None, None]
    out = nets.conv(xq, wq) * sc
    if not with_bound:
        return out
    return out, nets.conv(np.abs(xq), np.abs(wq)) * sc


def accumulation_bound(abs_sum, k):
    """Worst-case error of a float32 sum of k terms (recursive summation,
    k * 2^-24 relative to the sum of magnitudes), plus the rounding of the
    final rescale."""
    return abs_sum * (k + 2) * 2.0 ** -24


def bf16_half_step(v):
    """Half the bfloat16 spacing at |v| (8 significant bits)."""
    a = np.maximum(np.abs(v), 2.0 ** -126)
    return np.exp2(np.floor(np.log2(a)) - 8)


def synthesis_fp8(y_hat, wts, T, H, W):
    """Frames (T, 3, H, W) through the FP8 synthesis path."""
    a = bf16(nets.relu(nets.conv(bf16(y_hat), bf16(wts["d1"]))))
    for name in ("d2", "d3"):
        a = bf16(nets.relu(fp8_conv(a, a.max(), wts[name])))
    F, famax = a, a.max()
    g1 = [bf16(nets.relu(fp8_conv(F, famax, wts[f"k1_{t}"]))) for t in range(T)]
    amax1 = max(g.max() for g in g1)
    g2 = [bf16(nets.relu(fp8_conv(g, amax1, wts[f"k2_{t}"]))) for t, g in enumerate(g1)]
    amax2 = max(g.max() for g in g2)
    out = np.empty((T, 3, H, W))
    for t in range(T):
        o = fp8_conv(g2[t], amax2, wts[f"k3_{t}"])
        out[t] = np.clip(nets.pixel_shuffle8(o)[:, :H, :W], 0.0, 1.0)
    return out
