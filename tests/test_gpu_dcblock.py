"""GPU parity of the fused DC block (supplementary DC-block section; the
structure read as t = relu(pw1 x), x1 = x + pw2 dw3x3(t),
y = x1 + pw4 relu(pw3 x1)) against the float64 oracle, whole tensors,
through the C ABI.

The kernel computes in bf16 with float32 accumulation and rounds four
intermediate tensors to bf16 (each a relative step of at most 2^-9), so the
bar is relative to the output's scale: max abs <= 2% of max |y| and mean
abs <= 0.5% of mean |y| (both printed).  Sizes span one tile, ragged edge
tiles, a single position, and the 1080p latent (136 x 240) at C = 128.
The input is the bf16-rounded feature map, fed identically to both sides.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import dcblock  # noqa: E402
from synthetic import dc_block_weights, feature_map  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("C,h,w", [(64, 8, 16), (64, 18, 26), (128, 1, 1), (128, 3, 5),
                                   (128, 18, 26), (128, 136, 240)])
def test_dc_block_matches_oracle(C, h, w):
    import paper_2606_04410_amd as u
    say(f"dc block C={C} {h}x{w}")
    wt = dc_block_weights(C, seed=1)
    x32 = torch.from_numpy(np.ascontiguousarray(np.transpose(feature_map(C, h, w, seed=3), (1, 2, 0))))
    xb = x32.to(torch.bfloat16)
    blk = u.DcBlock(C, wt)
    try:
        y = blk.run(xb.cuda()).float().cpu().numpy()
    finally:
        blk.close()
    x64 = np.transpose(xb.float().numpy().astype(np.float64), (2, 0, 1))
    ref = np.transpose(dcblock.dc_block(x64, wt), (1, 2, 0))
    err = np.abs(y - ref)
    say(f"  max abs {err.max():.3e} (max |y| {np.abs(ref).max():.2f}), mean abs {err.mean():.3e} "
        f"(mean |y| {np.abs(ref).mean():.3f})")
    assert np.isfinite(y).all()
    assert err.max() <= 0.02 * np.abs(ref).max()
    assert err.mean() <= 0.005 * np.abs(ref).mean()


def test_dc_block_argument_errors():
    import paper_2606_04410_amd as u
    wt = dc_block_weights(64, seed=1)
    with pytest.raises(u.UfvcError):
        u.DcBlock(96, dc_block_weights(96))
    blk = u.DcBlock(64, wt)
    try:
        x = torch.zeros((4, 4, 64), dtype=torch.bfloat16, device="cuda")
        assert u.lib.ufvc_dcblock_run(blk._h, x.data_ptr(), x.data_ptr(), 4, 4, None) == -1
        assert u.lib.ufvc_dcblock_run(blk._h, x.data_ptr(), x.data_ptr() + 2048, 0, 4, None) == -1
    finally:
        blk.close()
