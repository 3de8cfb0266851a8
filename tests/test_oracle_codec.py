"""End-to-end oracle pins: container, round trip, golden bit-stream."""
import hashlib
import os

import numpy as np
import pytest

from oracle import codec, container, entropy, rans
from synthetic import stand_in_weights, video_chunk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_container_round_trip_and_errors():
    z = [b"\1" * 128, b"\2" * 132]
    y = [b"\3" * 136]
    bs = container.pack(4, 64, 64, 64, 14, 10, 22, 0xDEADBEEF, z, y)
    d = container.parse(bs)
    assert (d["T"], d["C"], d["H"], d["W"], d["seg_log2"], d["seg_log2_z"], d["k_z"],
            d["model_tag"]) == (4, 64, 64, 64, 14, 10, 22, 0xDEADBEEF)
    assert d["z_segs"] == z and d["y_segs"] == y
    assert bs[:4] == b"UFV1" and len(bs) == 28 + 12 + 128 + 132 + 136
    for bad in (bs[:20], bs[:-1], bs + b"\0\0\0\0", b"XFV1" + bs[4:]):
        with pytest.raises(container.BadContainer):
            container.parse(bad)
    # the flags byte: the quadtree bit round-trips, unknown bits are refused
    assert d["flags"] == 0
    q = container.pack(4, 64, 64, 64, 14, 10, 22, 1, z, y, flags=container.FLAG_QUADTREE)
    assert q[15] == 1 and container.parse(q)["flags"] == container.FLAG_QUADTREE
    with pytest.raises(container.BadContainer):
        container.parse(q[:15] + b"\x04" + q[16:])


@pytest.fixture(scope="module")
def c1():
    fr = video_chunk(4, 64, 64, 3, seed=1)
    w = stand_in_weights(4, 64)
    bs, inter = codec.encode_chunk(fr, w, seg_log2=14, seg_log2_z=10, model_tag=0x55F00401)
    return fr, w, bs, inter


def test_c1_round_trip(c1):
    fr, w, bs, enc = c1
    x_hat, dec = codec.decode_chunk(bs, w)
    np.testing.assert_array_equal(dec["y_sym"], enc["y_sym"])
    np.testing.assert_array_equal(dec["idx"], enc["idx"])
    np.testing.assert_array_equal(dec["z_hat"], enc["z_hat"])
    assert x_hat.shape == fr.shape and x_hat.min() >= 0 and x_hat.max() <= 1
    # y_hat = r_hat + mu, with r_hat = round(y - mu)
    assert np.all(np.abs(dec["y_hat"] - enc["y"]) <= 0.5 + 1e-9)


def test_c1_code_length(c1):
    _, _, bs, enc = c1
    d = container.parse(bs)
    payload_bits = 8 * sum(len(s) for s in d["z_segs"] + d["y_segs"])
    n_seg = len(d["z_segs"]) + len(d["y_segs"])
    ideal = enc["bits_ideal"]
    assert 0 <= payload_bits - ideal <= 0.005 * ideal + 32 * 32 * n_seg


def test_c1_golden_hash(c1):
    _, _, bs, _ = c1
    with open(os.path.join(GOLDEN, "c1_bitstream.sha256")) as f:
        want = f.read().split()[0]
    assert hashlib.sha256(bs).hexdigest() == want


def test_decoder_rejects_corruption(c1):
    _, w, bs, _ = c1
    with pytest.raises((rans.CorruptStream, container.BadContainer)):
        codec.decode_chunk(bs[:-8], w)
    bad = bytearray(bs)
    bad[len(bs) // 2] ^= 0xFF
    with pytest.raises(rans.CorruptStream):
        codec.decode_chunk(bytes(bad), w)


def test_scale_index_of_decoder_matches_encoder_exactly(c1):
    _, w, bs, enc = c1
    _, dec = codec.decode_latent(bs, w)
    assert np.array_equal(dec["idx"], entropy.scale_index(enc["sigma"]))


def test_psnr_closed_forms():
    """PSNR = 10 log10(1 / MSE) with peak 1: a uniform error d gives
    -20 log10 d; the same error on half the values adds 10 log10 2; identical
    inputs give infinity; the result does not depend on the array's shape."""
    a = np.zeros((2, 3, 8, 8))
    for d in (0.5, 0.1, 1e-3):
        assert abs(codec.psnr(a, a + d) - (-20.0 * np.log10(d))) < 1e-9
        b = a.copy()
        b[0] += d                      # half of the values
        assert abs(codec.psnr(a, b) - (-20.0 * np.log10(d) + 10.0 * np.log10(2.0))) < 1e-9
    assert abs(codec.psnr(a.reshape(6, 64), (a + 0.1).reshape(6, 64)) - 20.0) < 1e-9
    assert codec.psnr(a + 0.3, a + 0.3) == float("inf")
    # symmetric in its arguments, and float32 inputs are promoted
    r = np.random.default_rng(0).random((3, 5)).astype(np.float32)
    assert codec.psnr(r, r * 0.5) == codec.psnr(r * 0.5, r)
