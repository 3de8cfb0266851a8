"""Stand-in neural transforms, float64, channel-first (C, H, W) arrays.

Test infrastructure only (see the package docstring).

The paper's pipeline (Sec. 3.1, Fig. 3): patch embedding to 1/8 resolution,
a chunk encoder producing one latent y for the whole chunk, a hyper prior
z_hat, an entropy-parameter network fed by the prior (Sec. 3.4), a chunk
decoder producing the joint feature F, then N frame-specific decoders, one per
temporal position (Sec. 3.2).  The stand-in replaces every DC block stack by
plain 3x3 convolutions with seeded random weights:

  analysis   X = patchify(pad(frames));  a1 = relu(conv(X)); a2 = relu(conv(a1));
             y = conv(a2)                                   (linear, signed)
  hyper      z = conv_stride2(y);  z_hat = clamp(rint(z), -32, 32)
  params     P = conv(up2(z_hat));  mu = P[:C];  sigma = clamp(softplus(P[C:]), 0.11, 64)
  synthesis  F = relu(conv(relu(conv(relu(conv(y_hat))))))  (cross-frame stack)
             o_t = conv(relu(conv(relu(conv(F, k1_t)), k2_t)), k3_t)
             x_hat_t = clamp(crop(pixel_shuffle8(o_t)), 0, 1)

Temporal chunk context (Sec. 3.1 with the Fig. 2 caption, Sec. 3.3, Sec. 3.4):
a model whose weights hold the context layers (c1, c2, a1c, pc, d1c) carries
the context C_i of chunk i.  It conditions the chunk encoder (a1 also sees
C_i), the prior s_i of the entropy parameters (P also sees C_i) and the chunk
decoder (d1 also sees C_i); each "also sees" is a concatenation along
channels, i.e. one more conv summed in before the activation.  The joint
feature F_i of chunk i forms the next context through the context network,
C_{i+1} = relu(conv(relu(conv(F_i, c1)), c2)); the first chunk of a stream
has C_0 = 0 (so it is coded exactly as by the base model).  The paper gives
no internals (readings).

Pins: ``conv`` against a brute-force seven-loop sum and torch's float64
conv2d; ``patchify`` / ``pixel_shuffle8`` / ``up2`` / ``pad16`` against torch's
pixel_unshuffle / pixel_shuffle / nearest interpolate / replicate pad;
``softplus`` against its closed form at special points and torch; the
composed transforms against the same composition written with torch.nn
functional routines.
"""
from __future__ import annotations

import numpy as np

SIGMA_MIN = 0.11
SIGMA_MAX = 64.0
RMAX = 32  # symbols live in [-32, 32]


def padded_size(H: int, W: int) -> tuple[int, int]:
    """Frames are padded up to a multiple of 16 so the latent (1/8) is even."""
    return -(-H // 16) * 16, -(-W // 16) * 16


def pad16(frames: np.ndarray) -> np.ndarray:
    """Edge-replicate (T, 3, H, W) frames up to multiples of 16 in H and W."""
    T, c, H, W = frames.shape
    Hp, Wp = padded_size(H, W)
    rows = np.minimum(np.arange(Hp), H - 1)
    cols = np.minimum(np.arange(Wp), W - 1)
    return frames[:, :, rows][:, :, :, cols]


def patchify(frames_padded: np.ndarray) -> np.ndarray:
    """Pixel-unshuffle by 8 per frame, concatenated over time.

    X[t*192 + c*64 + i*8 + j, v, u] = frame[t, c, 8v + i, 8u + j]
    (the 1/8-resolution patch embedding of Sec. 3.1).
    """
    T, c, Hp, Wp = frames_padded.shape
    h, w = Hp // 8, Wp // 8
    x = frames_padded.reshape(T, c, h, 8, w, 8)          # t c v i u j
    x = x.transpose(0, 1, 3, 5, 2, 4)                    # t c i j v u
    return np.ascontiguousarray(x.reshape(T * c * 64, h, w), dtype=np.float64)


def pixel_shuffle8(o: np.ndarray) -> np.ndarray:
    """(192, h, w) -> (3, 8h, 8w): x[c, 8v+i, 8u+j] = o[c*64 + i*8 + j, v, u]."""
    _, h, w = o.shape
    x = o.reshape(3, 8, 8, h, w).transpose(0, 3, 1, 4, 2)  # c v i u j
    return x.reshape(3, 8 * h, 8 * w)


def conv(x: np.ndarray, wt: np.ndarray, stride: int = 1) -> np.ndarray:
    """3x3 convolution, zero padding 1, no bias, float64.

    out[o, v, u] = sum_{ky,kx,i} wt[o, i, ky, kx] * x[i, s*v + ky - 1, s*u + kx - 1]

    One tensordot per tap (BLAS does the channel sum); nothing else is
    reordered.
    """
    cin, H, W = x.shape
    cout = wt.shape[0]
    assert wt.shape == (cout, cin, 3, 3)
    Ho = (H - 1) // stride + 1
    Wo = (W - 1) // stride + 1
    xp = np.zeros((cin, H + 2, W + 2), dtype=np.float64)
    xp[:, 1:H + 1, 1:W + 1] = x
    w64 = wt.astype(np.float64)
    out = np.zeros((cout, Ho, Wo), dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride,
                       kx:kx + stride * (Wo - 1) + 1:stride]
            out += np.tensordot(w64[:, :, ky, kx], patch, axes=(1, 0))
    return out


def relu(x: np.ndarray) -> np.ndarray:
    return np.maximum(x, 0.0)


def softplus(x: np.ndarray) -> np.ndarray:
    """log(1 + e^x), evaluated as max(x, 0) + log1p(exp(-|x|))."""
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def up2(z: np.ndarray, h: int, w: int) -> np.ndarray:
    """Nearest-neighbour upsampling by 2, cropped to (h, w)."""
    return np.repeat(np.repeat(z, 2, axis=1), 2, axis=2)[:, :h, :w]


def rint_clamp(x: np.ndarray) -> np.ndarray:
    """Round half to even, then clamp to the coded range [-32, 32]."""
    return np.clip(np.rint(x), -RMAX, RMAX)


def analysis(frames: np.ndarray, wts: dict, ctx: np.ndarray = None) -> np.ndarray:
    """Chunk encoder: frames (T, 3, H, W) in [0, 1] -> latent y (C, h, w);
    with a temporal context ctx (C, h, w), a1 sees concat(X, ctx)."""
    X = patchify(pad16(frames.astype(np.float64)))
    pre = conv(X, wts["a1"])
    if ctx is not None:
        pre = pre + conv(ctx, wts["a1c"])
    a1 = relu(pre)
    a2 = relu(conv(a1, wts["a2"]))
    return conv(a2, wts["a3"])


def hyper(y: np.ndarray, wts: dict) -> np.ndarray:
    """Hyper prior: z = stride-2 conv of y; returns z_hat = clamp(rint(z))."""
    return rint_clamp(conv(y, wts["h"], stride=2))


def params(z_hat: np.ndarray, wts: dict, h: int, w: int, ctx: np.ndarray = None):
    """Entropy parameters in one pass (Sec. 3.4): returns (mu, sigma).  With a
    temporal context the prior is s = concat(up2(z_hat), ctx)."""
    C = wts["p"].shape[0] // 2
    P = conv(up2(z_hat, h, w), wts["p"])
    if ctx is not None:
        P = P + conv(ctx, wts["pc"])
    mu = P[:C]
    sigma = np.clip(softplus(P[C:]), SIGMA_MIN, SIGMA_MAX)
    return mu, sigma


def chunk_decoder(y_hat: np.ndarray, wts: dict, ctx: np.ndarray = None) -> np.ndarray:
    """Cross-frame stack producing the joint feature F (Sec. 3.1); with a
    temporal context, d1 sees concat(y_hat, ctx)."""
    pre = conv(y_hat, wts["d1"])
    if ctx is not None:
        pre = pre + conv(ctx, wts["d1c"])
    f = relu(pre)
    f = relu(conv(f, wts["d2"]))
    return relu(conv(f, wts["d3"]))


def frame_decoder(F: np.ndarray, wts: dict, t: int, H: int, W: int) -> np.ndarray:
    """Frame-specific decoder for temporal position t (Sec. 3.2) -> (3, H, W)."""
    g = relu(conv(F, wts[f"k1_{t}"]))
    g = relu(conv(g, wts[f"k2_{t}"]))
    o = conv(g, wts[f"k3_{t}"])
    return np.clip(pixel_shuffle8(o)[:, :H, :W], 0.0, 1.0)


def context(F: np.ndarray, wts: dict) -> np.ndarray:
    """Temporal context of the next chunk from this chunk's joint feature."""
    return relu(conv(relu(conv(F, wts["c1"])), wts["c2"]))


def synthesis(y_hat: np.ndarray, wts: dict, T: int, H: int, W: int,
              clamp: bool = True, ctx: np.ndarray = None) -> np.ndarray:
    """Chunk decoder + T frame-specific decoders -> frames (T, 3, H, W)."""
    F = chunk_decoder(y_hat, wts, ctx)
    out = np.empty((T, 3, H, W), dtype=np.float64)
    for t in range(T):
        if clamp:
            out[t] = frame_decoder(F, wts, t, H, W)
        else:
            g = relu(conv(F, wts[f"k1_{t}"]))
            g = relu(conv(g, wts[f"k2_{t}"]))
            out[t] = pixel_shuffle8(conv(g, wts[f"k3_{t}"]))[:, :H, :W]
    return out
