"""Chunk encode / decode end to end, and metrics.

Test infrastructure only (see the package docstring).

encode (Sec. 3.1, 3.4): y = analysis(X); z_hat = hyper(y); (mu, sigma) =
params(z_hat) in one pass; idx = scale_index(sigma); r_hat = round(y - mu);
z_hat and r_hat are coded by rANS (z_hat with the fixed table row k_z and mean
0) in channels-innermost order n = (v w + u) C + c.

decode: parse; decode z_hat; recompute (mu, sigma, idx) from z_hat exactly as
the encoder did; decode all of r_hat in one step (its tables depend only on
sigma); y_hat = r_hat + mu; synthesis.

Models whose weights include the context layers (c1, c2, a1c, pc, d1c) code
every chunk conditioned on the temporal context of its stream (``ctx``, the
C_i of nets; zeros for a stream's first chunk): encode and decode return the
next chunk's context in their intermediates (``ctx_next``), formed from the
joint feature of the decoded latent, which the encoder therefore also
computes.  Their streams carry container.FLAG_TEMPORAL.

Models whose weights include the mean-step layers m1..m3 use the quadtree
progressive means (``quadtree``): the single pass gives every scale and the
base mean, partitions 1..3 get refined means one step at a time (encoder:
before quantising each partition; decoder: after the one-step decode).  Their
streams carry container.FLAG_QUADTREE.
"""
from __future__ import annotations

import numpy as np

from . import container, entropy, nets, quadtree, rans


def latent_size(H: int, W: int) -> tuple[int, int, int, int]:
    """(h, w, hz, wz): latent and hyper-latent spatial sizes."""
    Hp, Wp = nets.padded_size(H, W)
    h, w = Hp // 8, Wp // 8
    return h, w, -(-h // 2), -(-w // 2)


def to_hwc(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.transpose(a, (1, 2, 0))).reshape(-1)


def from_hwc(v: np.ndarray, c: int, h: int, w: int) -> np.ndarray:
    return np.transpose(np.asarray(v).reshape(h, w, c), (2, 0, 1))


def is_temporal(wts) -> bool:
    return "c1" in wts


def zero_context(wts, H: int, W: int) -> np.ndarray:
    """C_0: the context of a stream's first chunk."""
    h, w, _, _ = latent_size(H, W)
    return np.zeros((wts["a2"].shape[0], h, w))


def encode_chunk(frames, wts, seg_log2=14, seg_log2_z=10, model_tag=0, tables=None, ctx=None):
    """Returns (bitstream bytes, dict of intermediates).  Temporal models take
    the stream's context ctx (default: a first chunk's zeros)."""
    T, _, H, W = frames.shape
    C = wts["a2"].shape[0]
    h, w, hz, wz = latent_size(H, W)
    freq, cum = tables if tables is not None else entropy.cdf_tables()
    if is_temporal(wts) and ctx is None:
        ctx = zero_context(wts, H, W)
    if not is_temporal(wts):
        ctx = None
    y = nets.analysis(frames, wts, ctx)
    z_hat = nets.hyper(y, wts)
    mu, sigma = nets.params(z_hat, wts, h, w, ctx)
    idx = entropy.scale_index(sigma)
    flags = 0
    if "m1" in wts:
        mu_base = mu
        mu, r_hat = quadtree.encode_means(y, mu_base, wts)
        sym = (r_hat + 32).astype(np.uint8)
        flags |= container.FLAG_QUADTREE
    else:
        sym = entropy.symbolise(y, mu)
    inter_t = {}
    if ctx is not None:
        flags |= container.FLAG_TEMPORAL
        y_hat = sym.astype(np.float64) - 32.0 + mu
        F = nets.chunk_decoder(y_hat, wts, ctx)
        inter_t = dict(F=F, ctx=ctx, ctx_next=nets.context(F, wts))
    z_sym = to_hwc(z_hat + 32).astype(np.uint8)
    y_sym = to_hwc(sym)
    y_idx = to_hwc(idx)
    z_segs = rans.encode(z_sym, np.full(z_sym.size, entropy.K_Z), freq, cum, 1 << seg_log2_z)
    y_segs = rans.encode(y_sym, y_idx, freq, cum, 1 << seg_log2)
    bs = container.pack(T, C, H, W, seg_log2, seg_log2_z, entropy.K_Z, model_tag, z_segs, y_segs,
                        flags)
    inter = dict(y=y, z_hat=z_hat, mu=mu, sigma=sigma, idx=idx, y_sym=y_sym, y_idx=y_idx,
                 z_sym=z_sym, bits_ideal=entropy.ideal_bits(y_sym, y_idx, freq)
                 + entropy.ideal_bits(z_sym, np.full(z_sym.size, entropy.K_Z), freq), **inter_t)
    return bs, inter


def decode_latent(bs: bytes, wts, tables=None, ctx=None):
    """Bit-stream -> (header dict, z_hat, mu, sigma, idx, y_sym (HWC), y_hat)."""
    hdr = container.parse(bs)
    C = wts["a2"].shape[0]
    if hdr["C"] != C:
        raise container.BadContainer("channel count mismatch")
    if bool(hdr["flags"] & container.FLAG_TEMPORAL) != is_temporal(wts):
        raise container.BadContainer("stream and model disagree on the temporal context")
    if is_temporal(wts) and ctx is None:
        ctx = zero_context(wts, hdr["H"], hdr["W"])
    if not is_temporal(wts):
        ctx = None
    if bool(hdr["flags"] & container.FLAG_QUADTREE) != ("m1" in wts):
        raise container.BadContainer("stream and model disagree on the mean estimation")
    freq, cum = tables if tables is not None else entropy.cdf_tables()
    h, w, hz, wz = latent_size(hdr["H"], hdr["W"])
    nz = hz * wz * 32
    z_sym = rans.decode(hdr["z_segs"], np.full(nz, hdr["k_z"]), freq, cum, 1 << hdr["seg_log2_z"])
    z_hat = from_hwc(z_sym.astype(np.float64) - 32.0, 32, hz, wz)
    mu, sigma = nets.params(z_hat, wts, h, w, ctx)
    idx = entropy.scale_index(sigma)
    y_idx = to_hwc(idx)
    y_sym = rans.decode(hdr["y_segs"], y_idx, freq, cum, 1 << hdr["seg_log2"])
    r_hat = from_hwc(y_sym.astype(np.float64) - 32.0, C, h, w)
    if "m1" in wts:
        mu = quadtree.decode_means(r_hat, mu, wts)
    y_hat = r_hat + mu
    return hdr, dict(z_hat=z_hat, mu=mu, sigma=sigma, idx=idx, y_idx=y_idx, y_sym=y_sym,
                     y_hat=y_hat, ctx=ctx)


def decode_chunk(bs: bytes, wts, tables=None, ctx=None):
    """Returns (frames (T, 3, H, W) float64, dict of intermediates); temporal
    models also return the next chunk's context as ctx_next."""
    hdr, inter = decode_latent(bs, wts, tables, ctx)
    T, H, W = hdr["T"], hdr["H"], hdr["W"]
    F = nets.chunk_decoder(inter["y_hat"], wts, inter["ctx"])
    x_hat = np.empty((T, 3, H, W))
    for t in range(T):
        x_hat[t] = nets.frame_decoder(F, wts, t, H, W)
    if inter["ctx"] is not None:
        inter["F"] = F
        inter["ctx_next"] = nets.context(F, wts)
    return x_hat, inter


def encode_sequence(chunks, wts, **kw):
    """Chunks of one stream in order: each coded with the context the
    previous one left (a temporal model), or independently.  Returns the
    streams and the intermediates."""
    ctx, out = None, []
    for fr in chunks:
        bs, inter = encode_chunk(fr, wts, ctx=ctx, **kw)
        ctx = inter.get("ctx_next")
        out.append((bs, inter))
    return out


def decode_sequence(streams, wts, tables=None):
    """Inverse of encode_sequence, in stream order."""
    ctx, out = None, []
    for bs in streams:
        x_hat, inter = decode_chunk(bs, wts, tables, ctx)
        ctx = inter.get("ctx_next")
        out.append((x_hat, inter))
    return out


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
