"""Chunk encode / decode end to end, and metrics.

Test infrastructure only (see the package docstring).

encode (Sec. 3.1, 3.4): y = analysis(X); z_hat = hyper(y); (mu, sigma) =
params(z_hat) in one pass; idx = scale_index(sigma); r_hat = round(y - mu);
z_hat and r_hat are coded by rANS (z_hat with the fixed table row k_z and mean
0) in channels-innermost order n = (v w + u) C + c.

decode: parse; decode z_hat; recompute (mu, sigma, idx) from z_hat exactly as
the encoder did; decode all of r_hat in one step (its tables depend only on
sigma); y_hat = r_hat + mu; synthesis.

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


def encode_chunk(frames, wts, seg_log2=14, seg_log2_z=10, model_tag=0, tables=None):
    """Returns (bitstream bytes, dict of intermediates)."""
    T, _, H, W = frames.shape
    C = wts["a2"].shape[0]
    h, w, hz, wz = latent_size(H, W)
    freq, cum = tables if tables is not None else entropy.cdf_tables()
    y = nets.analysis(frames, wts)
    z_hat = nets.hyper(y, wts)
    mu, sigma = nets.params(z_hat, wts, h, w)
    idx = entropy.scale_index(sigma)
    flags = 0
    if "m1" in wts:
        mu_base = mu
        mu, r_hat = quadtree.encode_means(y, mu_base, wts)
        sym = (r_hat + 32).astype(np.uint8)
        flags |= container.FLAG_QUADTREE
    else:
        sym = entropy.symbolise(y, mu)
    z_sym = to_hwc(z_hat + 32).astype(np.uint8)
    y_sym = to_hwc(sym)
    y_idx = to_hwc(idx)
    z_segs = rans.encode(z_sym, np.full(z_sym.size, entropy.K_Z), freq, cum, 1 << seg_log2_z)
    y_segs = rans.encode(y_sym, y_idx, freq, cum, 1 << seg_log2)
    bs = container.pack(T, C, H, W, seg_log2, seg_log2_z, entropy.K_Z, model_tag, z_segs, y_segs,
                        flags)
    inter = dict(y=y, z_hat=z_hat, mu=mu, sigma=sigma, idx=idx, y_sym=y_sym, y_idx=y_idx,
                 z_sym=z_sym, bits_ideal=entropy.ideal_bits(y_sym, y_idx, freq)
                 + entropy.ideal_bits(z_sym, np.full(z_sym.size, entropy.K_Z), freq))
    return bs, inter


def decode_latent(bs: bytes, wts, tables=None):
    """Bit-stream -> (header dict, z_hat, mu, sigma, idx, y_sym (HWC), y_hat)."""
    hdr = container.parse(bs)
    C = wts["a2"].shape[0]
    if hdr["C"] != C:
        raise container.BadContainer("channel count mismatch")
    if bool(hdr["flags"] & container.FLAG_QUADTREE) != ("m1" in wts):
        raise container.BadContainer("stream and model disagree on the mean estimation")
    freq, cum = tables if tables is not None else entropy.cdf_tables()
    h, w, hz, wz = latent_size(hdr["H"], hdr["W"])
    nz = hz * wz * 32
    z_sym = rans.decode(hdr["z_segs"], np.full(nz, hdr["k_z"]), freq, cum, 1 << hdr["seg_log2_z"])
    z_hat = from_hwc(z_sym.astype(np.float64) - 32.0, 32, hz, wz)
    mu, sigma = nets.params(z_hat, wts, h, w)
    idx = entropy.scale_index(sigma)
    y_idx = to_hwc(idx)
    y_sym = rans.decode(hdr["y_segs"], y_idx, freq, cum, 1 << hdr["seg_log2"])
    r_hat = from_hwc(y_sym.astype(np.float64) - 32.0, C, h, w)
    if "m1" in wts:
        mu = quadtree.decode_means(r_hat, mu, wts)
    y_hat = r_hat + mu
    return hdr, dict(z_hat=z_hat, mu=mu, sigma=sigma, idx=idx, y_idx=y_idx, y_sym=y_sym,
                     y_hat=y_hat)


def decode_chunk(bs: bytes, wts, tables=None):
    """Returns (frames (T, 3, H, W) float64, dict of intermediates)."""
    hdr, inter = decode_latent(bs, wts, tables)
    x_hat = nets.synthesis(inter["y_hat"], wts, hdr["T"], hdr["H"], hdr["W"])
    return x_hat, inter


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
