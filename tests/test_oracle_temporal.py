"""Pins for the temporal chunk context (Sec. 3.1, Fig. 2 caption; Sec. 3.3;
Sec. 3.4's prior s_i from z_hat and C_i), independent of the oracle's own
formulas: the context's concatenations written as torch convs over
concatenated tensors, the first chunk reducing to the base model, the
context network at zero, and encoder/decoder agreement over a sequence."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import codec, container, nets
from synthetic import stand_in_weights, video_chunk

T, H, W, C = 2, 32, 48, 16


def _wts():
    return stand_in_weights(T, C, temporal=True)


def _t(a):
    return torch.from_numpy(np.asarray(a, np.float64))


def test_context_conditioning_is_a_channel_concatenation():
    wts = _wts()
    rng = np.random.default_rng(1)
    h, w = 4, 6
    ctx = rng.standard_normal((C, h, w))
    fr = video_chunk(T, H, W, 3, seed=2)
    # a1 over concat(X, ctx) with the concatenated weight tensor
    X = nets.patchify(nets.pad16(fr.astype(np.float64)))
    wcat = np.concatenate([wts["a1"], wts["a1c"]], axis=1)
    a1 = F.relu(F.conv2d(torch.cat([_t(X), _t(ctx)])[None], _t(wcat), padding=1))[0]
    a2 = F.relu(F.conv2d(a1[None], _t(wts["a2"]), padding=1))[0]
    y = F.conv2d(a2[None], _t(wts["a3"]), padding=1)[0].numpy()
    np.testing.assert_allclose(nets.analysis(fr, wts, ctx), y, rtol=1e-10, atol=1e-10)
    # the prior: concat(up2(z_hat), ctx)
    z_hat = np.rint(rng.standard_normal((32, 2, 3)) * 3)
    up = np.repeat(np.repeat(z_hat, 2, 1), 2, 2)[:, :h, :w]
    pcat = np.concatenate([wts["p"], wts["pc"]], axis=1)
    P = F.conv2d(torch.cat([_t(up), _t(ctx)])[None], _t(pcat), padding=1)[0].numpy()
    mu, sigma = nets.params(z_hat, wts, h, w, ctx)
    np.testing.assert_allclose(mu, P[:C], rtol=1e-10, atol=1e-10)
    sp = np.clip(F.softplus(torch.from_numpy(P[C:])).numpy(), 0.11, 64)
    np.testing.assert_allclose(sigma, sp, rtol=1e-8, atol=1e-8)
    # d1 over concat(y_hat, ctx)
    y_hat = rng.standard_normal((C, h, w))
    dcat = np.concatenate([wts["d1"], wts["d1c"]], axis=1)
    f = F.relu(F.conv2d(torch.cat([_t(y_hat), _t(ctx)])[None], _t(dcat), padding=1))[0]
    f = F.relu(F.conv2d(f[None], _t(wts["d2"]), padding=1))[0]
    f = F.relu(F.conv2d(f[None], _t(wts["d3"]), padding=1))[0].numpy()
    np.testing.assert_allclose(nets.chunk_decoder(y_hat, wts, ctx), f, rtol=1e-10, atol=1e-10)
    # the context network
    c = F.relu(F.conv2d(F.relu(F.conv2d(_t(f)[None], _t(wts["c1"]), padding=1)), _t(wts["c2"]),
                        padding=1))[0].numpy()
    np.testing.assert_allclose(nets.context(f, wts), c, rtol=1e-10, atol=1e-10)


def test_first_chunk_equals_the_base_model():
    """C_0 = 0: the first chunk's stream is the base model's, bit for bit
    (the base layers' draws are unchanged), apart from the flag byte."""
    wts = _wts()
    base = stand_in_weights(T, C)
    for k in base:
        np.testing.assert_array_equal(base[k], wts[k])
    fr = video_chunk(T, H, W, 3, seed=3)
    bs_t, it = codec.encode_chunk(fr, wts, seg_log2=9, seg_log2_z=8)
    bs_b, ib = codec.encode_chunk(fr, base, seg_log2=9, seg_log2_z=8)
    assert bs_t[15] == container.FLAG_TEMPORAL and bs_b[15] == 0
    assert bs_t[:15] + bs_t[16:] == bs_b[:15] + bs_b[16:]
    np.testing.assert_array_equal(nets.context(np.zeros((C, 4, 6)), wts), 0.0)


def test_sequence_round_trip_and_context_agreement():
    wts = _wts()
    chunks = [video_chunk(T, H, W, 3, seed=4, chunk_id=k) for k in range(3)]
    enc = codec.encode_sequence(chunks, wts, seg_log2=9, seg_log2_z=8)
    dec = codec.decode_sequence([bs for bs, _ in enc], wts)
    for k, ((bs, ie), (x_hat, idd)) in enumerate(zip(enc, dec)):
        np.testing.assert_array_equal(idd["y_sym"], ie["y_sym"])
        np.testing.assert_array_equal(idd["y_idx"], ie["y_idx"])
        # the decoder's context equals the encoder's, chunk after chunk
        np.testing.assert_array_equal(idd["ctx"], ie["ctx"])
        np.testing.assert_array_equal(idd["ctx_next"], ie["ctx_next"])
        assert x_hat.shape == (T, 3, H, W)
        if k > 0:
            assert np.abs(ie["ctx"]).max() > 0     # later chunks see a real context
    # a chunk decoded with the wrong context gets other scales: its rANS
    # integrity check fails (or, had it passed, the latent would differ)
    from oracle import rans
    try:
        _, wrong = codec.decode_latent(enc[2][0], wts, ctx=enc[0][1]["ctx_next"])
    except rans.CorruptStream:
        wrong = None
    assert wrong is None or not np.array_equal(wrong["y_idx"], enc[2][1]["y_idx"])


def test_flag_mismatch_is_refused():
    wts = _wts()
    base = stand_in_weights(T, C)
    fr = video_chunk(T, H, W, 3, seed=5)
    bs_t, _ = codec.encode_chunk(fr, wts, seg_log2=9, seg_log2_z=8)
    with pytest.raises(container.BadContainer):
        codec.decode_latent(bs_t, base)
    bs_b, _ = codec.encode_chunk(fr, base, seg_log2=9, seg_log2_z=8)
    with pytest.raises(container.BadContainer):
        codec.decode_latent(bs_b, wts)
