"""GPU parity of the quadtree progressive means (Sec. 3.4, Fig. 3 (a)) against
the oracle, through the C ABI.

Each stage is isolated on the GPU's own inputs: the oracle's means are
computed from the GPU's z_hat (single pass) and the GPU's symbols (the three
steps), then

* means: every element within 1e-4 of the oracle's (float32 sums);
* symbols: round(y - mu) of the GPU's y and the oracle's mean, identical
  except within 1e-4 of a half-integer;
* container: byte-identical to the oracle's coding of the GPU's symbols and
  indices, with the quadtree flag;
* decoder: indices, symbols and the refined means identical to the
  encoder's, bit for bit (the same kernels in the same order);
* frames (float32): the oracle synthesis of y_hat = r_hat + mu within 1e-3;
* the oracle's own stream decodes on the GPU to the oracle's symbols wherever
  the indices agree, and a stream/model mismatch of the flag is refused.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import codec as ocodec  # noqa: E402
from oracle import container, entropy, nets, quadtree, rans  # noqa: E402
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


def run(prec, T, H, W, C, sl=13, slz=10, seed=1, shift=16, tag=0x0A7D_0001):
    say(f"quadtree {prec}: T={T} {W}x{H} C={C} seg {sl}/{slz}")
    w = stand_in_weights(T, C, quadtree=True)
    fr = video_chunk(T, H, W, shift, seed=seed)
    c = pkg().Codec(T, C, w, precision=prec, seg_log2=sl, seg_log2_z=slz, model_tag=tag,
                    autotune=(H >= 512))
    assert c.quadtree
    try:
        dfr = torch.from_numpy(fr).cuda()
        bs, n = c.encode(dfr)
        g_bs = bs[:n].cpu().numpy().tobytes()
        h, ww, hz, wz = c.latent_size(H, W)
        g_y = c.buffer(pkg().BUF_Y, H, W).astype(np.float64)
        g_z = c.buffer(pkg().BUF_ZSYM, H, W).astype(np.int64) - 32
        g_P = c.buffer(pkg().BUF_PARAMS, H, W)
        g_idx = c.buffer(pkg().BUF_IDX, H, W)
        g_sym = c.buffer(pkg().BUF_SYM, H, W)
        # oracle means from the GPU's z_hat and symbols
        mu_base, sigma = nets.params(chw(g_z).astype(np.float64), w, h, ww)
        r_gpu = chw(g_sym).astype(np.float64) - 32.0
        mu = hwc(quadtree.decode_means(r_gpu, mu_base, w))
        part = hwc(quadtree.partition(C, h, ww))
        dmu = np.abs(g_P[..., :C].astype(np.float64) - mu)
        say(f"  means: max abs {dmu.max():.3e} (partition 0: {dmu[part == 0].max():.3e}, "
            f"1-3: {dmu[part > 0].max():.3e}), |mu| max {np.abs(mu).max():.2f}")
        assert dmu.max() < 1e-4
        # symbols: round(y - mu) of the GPU's y and the oracle's mean
        r = g_y - mu
        o_sym = np.clip(np.rint(r), -32, 32) + 32
        smis = g_sym != o_sym
        say(f"  symbols: {int(smis.sum())} of {g_sym.size} differ, "
            f"{int(near_half(r).sum())} in the 1e-4 band")
        assert not (smis & ~near_half(r)).any()
        # scale indices: the single pass is unchanged by the quadtree
        imis = g_idx != hwc(entropy.scale_index(sigma))
        assert not (imis & ~near_threshold(hwc(sigma))).any()
        # the container: the oracle's coding of the GPU's symbols and indices
        zs = (g_z + 32).astype(np.uint8).reshape(-1)
        want = container.pack(T, C, H, W, sl, slz, entropy.K_Z, tag,
                              rans.encode(zs, np.full(zs.size, entropy.K_Z), FREQ, CUM, 1 << slz),
                              rans.encode(g_sym.reshape(-1), g_idx.reshape(-1), FREQ, CUM, 1 << sl),
                              container.FLAG_QUADTREE)
        assert g_bs == want
        say(f"  container: {n} bytes, byte-equal to the oracle's, flags {g_bs[15]}")
        # GPU decode: same indices, symbols and refined means as the encoder
        out = c.decode(bs, n, H, W)
        np.testing.assert_array_equal(c.buffer(pkg().BUF_IDX, H, W), g_idx)
        np.testing.assert_array_equal(c.buffer(pkg().BUF_SYM, H, W), g_sym)
        d_P = c.buffer(pkg().BUF_PARAMS, H, W)
        np.testing.assert_array_equal(d_P[..., :C].view(np.uint32), g_P[..., :C].view(np.uint32))
        x_hat = out.cpu().numpy()
        if prec == "fp32":
            y_hat = chw(g_sym.astype(np.float64) - 32.0 + d_P[..., :C].astype(np.float64))
            ref = nets.synthesis(y_hat, w, T, H, W)
            err = float(np.abs(x_hat - ref).max())
            say(f"  frames: max abs {err:.3e} vs the oracle synthesis of the GPU's y_hat")
            assert err <= 1e-3
        return c, w, fr, g_bs, g_idx
    except Exception:
        c.close()
        raise


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_quadtree_c1(prec):
    c, w, fr, g_bs, g_idx = run(prec, 4, 64, 64, 64, sl=10, slz=8, shift=3)
    try:
        # the oracle's own quadtree stream decodes on the GPU
        o_bs, o_inter = ocodec.encode_chunk(fr, w, seg_log2=10, seg_log2_z=8, model_tag=0x0A7D_0001)
        dev = torch.from_numpy(np.frombuffer(o_bs, np.uint8).copy()).cuda()
        c.decode(dev, len(o_bs), 64, 64, check=False)
        st = c.status()
        d_idx = c.buffer(pkg().BUF_IDX, 64, 64).reshape(-1)
        same = d_idx == o_inter["y_idx"]
        say(f"  oracle stream on the GPU: status {st}, index agreement {same.mean():.6f}")
        if same.all():
            assert st == 0
            np.testing.assert_array_equal(c.buffer(pkg().BUF_SYM, 64, 64).reshape(-1),
                                          o_inter["y_sym"])
        # a single-pass model refuses the quadtree stream (flag mismatch)
        plain = pkg().Codec(4, 64, stand_in_weights(4, 64), precision=prec, seg_log2=10,
                            seg_log2_z=8, model_tag=0x0A7D_0001)
        try:
            assert not plain.quadtree
            dbs = torch.from_numpy(np.frombuffer(g_bs, np.uint8).copy()).cuda()
            with pytest.raises(pkg().UfvcError) as e:
                plain.decode(dbs, len(g_bs), 64, 64)
            assert e.value.code == -1
            # and batches take single-pass models only
            with pytest.raises(pkg().UfvcError) as e:
                pkg().Batch([c])
            assert e.value.code == -6
        finally:
            plain.close()
    finally:
        c.close()


def test_quadtree_ragged_c128():
    """Several 16-column units per phase row with a ragged tail (latent
    18 x 26: 13 columns per phase), C = 128, float32."""
    c, *_ = run("fp32", 2, 144, 200, 128, sl=11, slz=9, seed=4)
    c.close()


def test_quadtree_1080p_whole_chunk_bf16():
    """Full size: every mean and symbol of a 1080p T = 8 chunk (C = 128)."""
    c, *_ = run("bf16", 8, 1080, 1920, 128, seed=1)
    try:
        c.profile(True)
        fr = torch.from_numpy(video_chunk(8, 1080, 1920, 16, seed=1)).cuda()
        bs, n = c.encode(fr)
        c.decode(bs, n, 1080, 1920)
        prof = c.profile_read()
        say("  mean steps per chunk: encoder %.1f us, decoder %.1f us (3 launches each)" % (
            1e3 * prof["mean_steps_enc"][0], 1e3 * prof["mean_steps_dec"][0]))
        c.profile(False)
    finally:
        c.close()
