"""GPU parity of the temporal chunk context (Sec. 3.1, Fig. 2 caption; the
prior s_i of Sec. 3.4) against the oracle, through the C ABI, over
sequences of chunks.

Each chunk's stages are isolated on the GPU's own inputs, the context
included (the oracle is handed the context the GPU's stream object holds):

* y: float32 max abs <= 1e-3; bf16 <= 2% of max |y|;
* z_hat, indices, symbols: identical except in the 1e-4 half-integer and
  1e-5 relative threshold bands; means within 1e-4 (the context's part of
  the entropy parameters is float32 arithmetic like the rest);
* the container: byte-identical to the oracle's coding of the GPU's
  symbols and indices, with the temporal flag;
* the next context: against the oracle's context network on the GPU's F
  (float32 1e-3; bf16 2% of max); the decoder's stream object ends every
  chunk with the encoder's context bit for bit, and the same symbols;
* float32 frames against the oracle synthesis of the GPU's y_hat and
  context within 1e-3;
* ufvc_encode_chunk refuses a temporal model; a NOSPC encode does not
  advance the context; reset gives zeros.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import container, entropy, nets, rans  # noqa: E402
from synthetic import stand_in_weights, video_chunk  # noqa: E402

FREQ, CUM = entropy.cdf_tables()
THR = entropy.thresholds().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pkg():
    import paper_2606_04410_amd as p
    return p


def hwc(a):
    return np.ascontiguousarray(np.transpose(a, (1, 2, 0)))


def chw(a):
    return np.ascontiguousarray(np.transpose(a, (2, 0, 1)))


def near_half(v, tol=1e-4):
    return np.abs(v - np.floor(v) - 0.5) < tol


def near_threshold(sigma, rel=1e-5):
    return (np.abs(sigma[..., None] - THR) / THR).min(axis=-1) < rel


def run_sequence(prec, T, H, W, C, n_chunks, sl, slz, shift, seed=1, tag=0x7E00_0001):
    u = pkg()
    w = stand_in_weights(T, C, temporal=True)
    c = u.Codec(T, C, w, precision=prec, seg_log2=sl, seg_log2_z=slz, model_tag=tag,
                autotune=(H >= 512))
    assert c.temporal
    enc, dec = u.Stream(c, H, W), u.Stream(c, H, W)
    h, ww, hz, wz = c.latent_size(H, W)
    y_tol = 1e-3 if prec == "fp32" else None
    try:
        for i in range(n_chunks):
            say(f"temporal {prec}: T={T} {W}x{H} C={C} chunk {i}")
            fr = video_chunk(T, H, W, shift, seed=seed, chunk_id=i)
            ctx = chw(enc.context()).astype(np.float64)
            if i == 0:
                assert not ctx.any()
            else:
                assert np.abs(ctx).max() > 0
            bs, n = enc.encode(torch.from_numpy(fr).cuda())
            g_bs = bs[:n].cpu().numpy().tobytes()
            g_y = c.buffer(u.BUF_Y, H, W).astype(np.float64)
            g_z = c.buffer(u.BUF_ZSYM, H, W).astype(np.int64) - 32
            g_P = c.buffer(u.BUF_PARAMS, H, W).astype(np.float64)
            g_idx = c.buffer(u.BUF_IDX, H, W)
            g_sym = c.buffer(u.BUF_SYM, H, W)
            g_F = chw(c.buffer(u.BUF_F, H, W)).astype(np.float64)
            nxt = enc.context()
            # analysis with the context
            o_y = hwc(nets.analysis(fr, w, ctx))
            ey = float(np.abs(g_y - o_y).max())
            assert ey <= (y_tol if y_tol else 0.02 * np.abs(o_y).max())
            # hyper on the GPU's y
            o_z = nets.conv(chw(g_y), w["h"], stride=2)
            zmis = g_z != hwc(nets.rint_clamp(o_z))
            assert not (zmis & ~near_half(hwc(o_z))).any()
            # entropy parameters from the GPU's z_hat and context
            mu, sigma = nets.params(chw(g_z).astype(np.float64), w, h, ww, ctx)
            dmu = float(np.abs(g_P[..., :C] - hwc(mu)).max())
            assert dmu < 1e-4
            imis = g_idx != hwc(entropy.scale_index(sigma))
            assert not (imis & ~near_threshold(hwc(sigma))).any()
            r = g_y - g_P[..., :C]
            smis = g_sym != np.clip(np.rint(r), -32, 32) + 32
            assert not (smis & ~near_half(r)).any()
            # the container
            zs = (g_z + 32).astype(np.uint8).reshape(-1)
            want = container.pack(T, C, H, W, sl, slz, entropy.K_Z, tag,
                                  rans.encode(zs, np.full(zs.size, entropy.K_Z), FREQ, CUM, 1 << slz),
                                  rans.encode(g_sym.reshape(-1), g_idx.reshape(-1), FREQ, CUM, 1 << sl),
                                  container.FLAG_TEMPORAL)
            assert g_bs == want
            # the next context from the GPU's F
            o_nxt = hwc(nets.context(g_F, w))
            ec = float(np.abs(nxt - o_nxt).max())
            assert ec <= (1e-3 if prec == "fp32" else 0.02 * max(np.abs(o_nxt).max(), 1e-6))
            # decoder: same symbols and indices, same next context bit for bit
            out = dec.decode(bs, n)
            np.testing.assert_array_equal(c.buffer(u.BUF_IDX, H, W), g_idx)
            np.testing.assert_array_equal(c.buffer(u.BUF_SYM, H, W), g_sym)
            np.testing.assert_array_equal(dec.context().view(np.uint32), nxt.view(np.uint32))
            msg = (f"  y {ey:.2e}, means {dmu:.2e}, {int(smis.sum())} symbols / {int(imis.sum())} "
                   f"indices in their bands, next context {ec:.2e} (max {np.abs(o_nxt).max():.2f}), "
                   f"{n} bytes")
            if prec == "fp32":
                y_hat = chw(g_sym.astype(np.float64) - 32.0 + g_P[..., :C])
                ref = nets.synthesis(y_hat, w, T, H, W, ctx=ctx)
                ef = float(np.abs(out.cpu().numpy() - ref).max())
                msg += f", frames {ef:.2e}"
                assert ef <= 1e-3
            say(msg)
        return c, enc, dec, w
    except Exception:
        enc.close()
        dec.close()
        c.close()
        raise


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_temporal_sequence_c1(prec):
    c, enc, dec, w = run_sequence(prec, 4, 64, 64, 64, 3, 10, 8, 3)
    u = pkg()
    try:
        # a temporal model codes only through stream objects
        fr = torch.from_numpy(video_chunk(4, 64, 64, 3, seed=1)).cuda()
        with pytest.raises(u.UfvcError) as e:
            c.encode(fr)
        assert e.value.code == -6
        # NOSPC leaves the context where it was
        before = enc.context()
        small = torch.empty(64, dtype=torch.uint8, device="cuda")
        with pytest.raises(u.UfvcError) as e:
            enc.encode(fr, out=small)
        assert e.value.code == -2
        np.testing.assert_array_equal(enc.context().view(np.uint32), before.view(np.uint32))
        # and the context of both sides tracks: one more chunk, then reset
        bs, n = enc.encode(fr)
        dec.decode(bs, n)
        np.testing.assert_array_equal(dec.context().view(np.uint32), enc.context().view(np.uint32))
        enc.reset()
        assert not enc.context().any()
        with pytest.raises(u.UfvcError):
            u.Stream(u.Codec(4, 64, stand_in_weights(4, 64), precision=prec), 64, 64)
    finally:
        enc.close()
        dec.close()
        c.close()


def test_temporal_sequence_ragged_c128_fp32():
    c, enc, dec, _ = run_sequence("fp32", 2, 144, 200, 128, 2, 11, 9, 16, seed=5)
    enc.close()
    dec.close()
    c.close()


def test_temporal_sequence_1080p_bf16():
    """Full size, whole tensors: two 1080p T = 8 chunks of one stream (the
    second coded with a real context)."""
    c, enc, dec, _ = run_sequence("bf16", 8, 1080, 1920, 128, 2, 13, 10, 16)
    enc.close()
    dec.close()
    c.close()
