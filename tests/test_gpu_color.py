"""GPU parity of the frame format conversions around the YUV444 interface
(supplementary RGB section; BT.709 full range, 4:2:0 by 2x2 repetition and
2x2 means) against the oracle, whole tensors, through the C ABI.

Bars: float32 arithmetic against float64, max abs <= 2e-6 on [0, 1] values
(4:2:0 -> 4:4:4 is a copy: bit-equal); in-place RGB <-> YUV444 equals
out-of-place; the codec's RGB and YUV420 paths equal converting on the GPU,
coding the YUV444 frames, and converting back; argument errors are refused.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import color  # noqa: E402
from synthetic import stand_in_weights, video_chunk  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pkg():
    import paper_2606_04410_amd as p
    return p


def flat420(y, cb, cr):
    T = y.shape[0]
    return np.concatenate([np.concatenate([y[t].ravel(), cb[t].ravel(), cr[t].ravel()])
                           for t in range(T)]).astype(np.float32)


def unflat420(v, T, H, W):
    v = np.asarray(v).reshape(T, -1)
    q = H * W // 4
    return (v[:, :H * W].reshape(T, H, W), v[:, H * W:H * W + q].reshape(T, H // 2, W // 2),
            v[:, H * W + q:].reshape(T, H // 2, W // 2))


@pytest.mark.parametrize("T,H,W", [(2, 64, 96), (1, 18, 20), (8, 1080, 1920)])
def test_conversions_match_oracle(T, H, W):
    say(f"colour conversions T={T} {W}x{H}")
    u = pkg()
    rgb = video_chunk(T, H, W, 3, seed=7)
    d = torch.from_numpy(rgb).cuda()
    yuv = u.convert_frames(d, "rgb", "yuv444", T, H, W)
    o_yuv = color.rgb_to_yuv444(rgb)
    e1 = float(np.abs(yuv.cpu().numpy() - o_yuv).max())
    back = u.convert_frames(yuv, "yuv444", "rgb", T, H, W)
    o_back = color.yuv444_to_rgb(yuv.cpu().numpy().astype(np.float64))
    e2 = float(np.abs(back.cpu().numpy() - o_back).max())
    e2r = float(np.abs(back.cpu().numpy() - rgb).max())
    # 4:2:0 both ways
    f420 = u.convert_frames(yuv, "yuv444", "yuv420", T, H, W)
    oy, ocb, ocr = color.yuv444_to_420(yuv.cpu().numpy().astype(np.float64))
    e3 = float(np.abs(f420.cpu().numpy() - flat420(oy, ocb, ocr)).max())
    full = u.convert_frames(f420, "yuv420", "yuv444", T, H, W)
    gy, gcb, gcr = unflat420(f420.cpu().numpy(), T, H, W)
    o_full = color.yuv420_to_444(gy, gcb, gcr).astype(np.float32)
    say(f"  rgb->yuv {e1:.2e}, yuv->rgb {e2:.2e} (round trip {e2r:.2e}), 444->420 {e3:.2e}")
    assert e1 <= 2e-6 and e2 <= 2e-6 and e3 <= 2e-6 and e2r <= 4e-6
    np.testing.assert_array_equal(full.cpu().numpy(), o_full)
    # in place: RGB <-> YUV444 on one buffer
    dd = d.clone()
    u.convert_frames(dd, "rgb", "yuv444", T, H, W, out=dd)
    np.testing.assert_array_equal(dd.cpu().numpy(), yuv.cpu().numpy())


def test_codec_rgb_and_yuv420_paths():
    say("codec rgb / yuv420 paths")
    u = pkg()
    T, H, W, C = 4, 64, 64, 64
    c = u.Codec(T, C, stand_in_weights(T, C), precision="fp32", seg_log2=12, seg_log2_z=10)
    try:
        rgb = torch.from_numpy(video_chunk(T, H, W, 3, seed=8)).cuda()
        yuv = u.convert_frames(rgb, "rgb", "yuv444", T, H, W)
        bs_a, na = c.encode(rgb, fmt="rgb")
        a = bs_a[:na].cpu().numpy().tobytes()
        bs_b, nb = c.encode(yuv)
        assert a == bs_b[:nb].cpu().numpy().tobytes()
        out_rgb = c.decode(bs_b, nb, H, W, fmt="rgb").cpu().numpy()
        out_yuv = c.decode(bs_b, nb, H, W)
        want = u.convert_frames(out_yuv, "yuv444", "rgb", T, H, W).cpu().numpy()
        np.testing.assert_array_equal(out_rgb, want)
        np.testing.assert_allclose(out_rgb, color.yuv444_to_rgb(out_yuv.cpu().numpy()), atol=2e-6)
        # YUV420 in, YUV420 out
        f420 = u.convert_frames(yuv, "yuv444", "yuv420", T, H, W)
        bs_c, nc = c.encode(f420, fmt="yuv420", H=H, W=W)
        full = u.convert_frames(f420, "yuv420", "yuv444", T, H, W)
        bs_d, nd = c.encode(full)
        assert bs_c[:nc].cpu().numpy().tobytes() == bs_d[:nd].cpu().numpy().tobytes()
        o420 = c.decode(bs_c, nc, H, W, fmt="yuv420").cpu().numpy()
        dy = c.decode(bs_c, nc, H, W).cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(o420, flat420(*color.yuv444_to_420(dy)), atol=2e-6)
    finally:
        c.close()


def test_conversion_argument_errors():
    u = pkg()
    x = torch.zeros((1, 3, 16, 16), device="cuda")
    y = torch.zeros((1, 3, 16, 16), device="cuda")
    lib = u.lib
    assert lib.ufvc_convert_frames(x.data_ptr(), 1, y.data_ptr(), 2, 1, 16, 16, None) == -6
    assert lib.ufvc_convert_frames(x.data_ptr(), 1, y.data_ptr(), 0, 1, 15, 16, None) == -1
    assert lib.ufvc_convert_frames(x.data_ptr(), 1, y.data_ptr(), 0, 1, 16, 14, None) == -1
    assert lib.ufvc_convert_frames(x.data_ptr(), 0, x.data_ptr(), 2, 1, 16, 16, None) == -1
    assert lib.ufvc_convert_frames(x.data_ptr(), 0, y.data_ptr(), 0, 1, 16, 16, None) == -6
    torch.cuda.synchronize()
