"""Edge sizes and argument errors through the C ABI.

* The smallest accepted frame (16x16: a 2x2 latent, one z position) and
  ragged sizes whose padding to 16 adds rows or columns: the container is
  byte-identical to the oracle coding the GPU's own symbols, the decoder
  recovers those symbols, and float32 frames match the oracle synthesis of
  the GPU's y_hat within 1e-3.
* Sizes the format excludes (under 16, not a multiple of 8) and short
  streams are refused with UFVC_E_INVAL before any kernel runs.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pkg():
    import paper_2606_04410_amd as p
    return p


@pytest.mark.parametrize("H,W", [(16, 16), (24, 40), (40, 24), (56, 72), (16, 200)])
def test_small_and_ragged_sizes_match_oracle(H, W):
    u = pkg()
    T, C = 4, 64
    say(f"edge size {H}x{W}")
    w = stand_in_weights(T, C)
    c = u.Codec(T, C, w, precision="fp32", seg_log2=8, seg_log2_z=5, model_tag=5)
    fr = video_chunk(T, H, W, 3, seed=H * 1000 + W)
    bs, n = c.encode(torch.from_numpy(fr).cuda())
    stream = bs[:n].cpu().numpy().tobytes()
    sym = c.buffer(u.BUF_SYM, H, W)
    idx = c.buffer(u.BUF_IDX, H, W)
    zs = c.buffer(u.BUF_ZSYM, H, W).reshape(-1)
    mu = c.buffer(u.BUF_PARAMS, H, W)[..., :C]
    z_segs = rans.encode(zs, np.full(zs.size, entropy.K_Z), FREQ, CUM, 1 << 5)
    y_segs = rans.encode(sym.reshape(-1), idx.reshape(-1), FREQ, CUM, 1 << 8)
    assert stream == container.pack(T, C, H, W, 8, 5, entropy.K_Z, 5, z_segs, y_segs)
    out = c.decode(bs, n, H, W).cpu().numpy()
    np.testing.assert_array_equal(c.buffer(u.BUF_SYM, H, W), sym)
    np.testing.assert_array_equal(c.buffer(u.BUF_IDX, H, W), idx)
    y_hat = np.transpose(sym.astype(np.float32) - 32 + mu, (2, 0, 1)).astype(np.float64)
    ref = nets.synthesis(y_hat, w, T, H, W)
    err = float(np.abs(out - ref).max())
    say(f"  {n} bytes, frames max abs {err:.2e}")
    assert out.shape == (T, 3, H, W) and err <= 1e-3
    c.close()


def test_sizes_outside_the_format_are_refused():
    u = pkg()
    T, C = 4, 64
    c = u.Codec(T, C, stand_in_weights(T, C), precision="bf16")
    for H, W in [(8, 64), (64, 8), (20, 64), (64, 36)]:
        fr = torch.zeros((T, 3, H, W), device="cuda")
        with pytest.raises(u.UfvcError) as e:
            c.encode(fr, out=torch.empty(1 << 16, dtype=torch.uint8, device="cuda"))
        assert e.value.code == -1, (H, W)
    bs = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(u.UfvcError) as e:
        c.decode(bs, 27, 64, 64)            # shorter than the header
    assert e.value.code == -1
    c.close()


@pytest.mark.parametrize("C,H,W", [(64, 64, 64), (128, 72, 136)])
def test_one_frame_chunks_match_oracle(C, H, W):
    """T = 1 (one-frame chunks, the chunk size of the paper's low-delay mode):
    the analysis conv runs on 192 input channels.  y matches the oracle's
    analysis, the container is byte-identical to the oracle coding the GPU's
    own symbols, the decoder recovers them, and the frames match the oracle
    synthesis of the GPU's y_hat."""
    u = pkg()
    T = 1
    say(f"one-frame chunk C={C} {H}x{W}")
    w = stand_in_weights(T, C)
    c = u.Codec(T, C, w, precision="fp32", seg_log2=10, seg_log2_z=7, model_tag=11, autotune=True)
    fr = video_chunk(T, H, W, 3, seed=C + H)
    bs, n = c.encode(torch.from_numpy(fr).cuda())
    stream = bs[:n].cpu().numpy().tobytes()
    y = c.buffer(u.BUF_Y, H, W)
    y_ref = np.transpose(nets.analysis(fr, w), (1, 2, 0))
    assert float(np.abs(y - y_ref).max()) <= 1e-3
    sym = c.buffer(u.BUF_SYM, H, W)
    idx = c.buffer(u.BUF_IDX, H, W)
    zs = c.buffer(u.BUF_ZSYM, H, W).reshape(-1)
    mu = c.buffer(u.BUF_PARAMS, H, W)[..., :C]
    z_segs = rans.encode(zs, np.full(zs.size, entropy.K_Z), FREQ, CUM, 1 << 7)
    y_segs = rans.encode(sym.reshape(-1), idx.reshape(-1), FREQ, CUM, 1 << 10)
    assert stream == container.pack(T, C, H, W, 10, 7, entropy.K_Z, 11, z_segs, y_segs)
    out = c.decode(bs, n, H, W).cpu().numpy()
    np.testing.assert_array_equal(c.buffer(u.BUF_SYM, H, W), sym)
    np.testing.assert_array_equal(c.buffer(u.BUF_IDX, H, W), idx)
    y_hat = np.transpose(sym.astype(np.float32) - 32 + mu, (2, 0, 1)).astype(np.float64)
    ref = nets.synthesis(y_hat, w, T, H, W)
    err = float(np.abs(out - ref).max())
    say(f"  {n} bytes, frames max abs {err:.2e}")
    assert out.shape == (T, 3, H, W) and err <= 1e-3
    c.close()
