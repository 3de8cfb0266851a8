"""Pins for the quadtree partition and the four-step progressive means
(Sec. 3.4, Fig. 3 (a)), independent of the oracle's own formulas: counting
and Latin-square properties of the partition, causality under perturbation,
a brute-force per-element neighbourhood sum, the zero-weight reduction to the
single pass, encoder/decoder agreement, and the end-to-end round trip."""
import itertools

import numpy as np
import pytest

from oracle import codec, container, nets, quadtree
from synthetic import stand_in_weights, video_chunk


@pytest.mark.parametrize("C,h,w", [(64, 8, 8), (128, 6, 10), (8, 4, 2)])
def test_partition_counts_and_latin_square(C, h, w):
    part = quadtree.partition(C, h, w)
    assert part.shape == (C, h, w)
    assert set(np.unique(part)) == {0, 1, 2, 3}
    # each partition is a quarter of the latent
    for k in range(4):
        assert (part == k).sum() == C * h * w // 4
    # at every position each partition holds exactly C / 4 channels (one group)
    for v, u in itertools.product(range(h), range(w)):
        counts = np.bincount(part[:, v, u], minlength=4)
        assert (counts == C // 4).all()
    # within a channel group, every 2x2 block holds each partition once
    for c in range(C):
        for v, u in itertools.product(range(0, h, 2), range(0, w, 2)):
            assert sorted(part[c, v:v + 2, u:u + 2].ravel()) == [0, 1, 2, 3]


def test_partition_phase_order_of_group_zero():
    # group 0 takes top-left, bottom-right, top-right, bottom-left in that order
    part = quadtree.partition(4, 2, 2)
    assert part[0, 0, 0] == 0 and part[0, 1, 1] == 1 and part[0, 0, 1] == 2 and part[0, 1, 0] == 3
    # the next channel group is shifted by one step
    assert part[1, 0, 0] == 1 and part[1, 1, 1] == 2


def _weights(C, seed):
    rng = np.random.default_rng(seed)
    return {f"m{k}": (rng.standard_normal((C, C, 3, 3)) * 0.1).astype(np.float32) for k in (1, 2, 3)}


def test_means_are_causal():
    """The mean of partition k depends on the residuals of partitions < k only."""
    C, h, w = 8, 6, 6
    rng = np.random.default_rng(1)
    wts = _weights(C, 2)
    mu_base = rng.standard_normal((C, h, w))
    r = np.rint(rng.standard_normal((C, h, w)) * 3)
    part = quadtree.partition(C, h, w)
    mu = quadtree.decode_means(r, mu_base, wts)
    for k in range(4):
        r2 = r.copy()
        later = part >= k
        r2[later] += rng.integers(-5, 6, later.sum())
        mu2 = quadtree.decode_means(r2, mu_base, wts)
        np.testing.assert_array_equal(mu2[part == k], mu[part == k])
    # partition 0 keeps the single pass's mean
    np.testing.assert_array_equal(mu[part == 0], mu_base[part == 0])


def test_means_bruteforce_neighbourhood_sum():
    C, h, w = 4, 4, 6
    rng = np.random.default_rng(3)
    wts = _weights(C, 4)
    mu_base = rng.standard_normal((C, h, w))
    r = np.rint(rng.standard_normal((C, h, w)) * 2)
    part = quadtree.partition(C, h, w)
    mu = quadtree.decode_means(r, mu_base, wts)
    for c, v, u in itertools.product(range(C), range(h), range(w)):
        k = part[c, v, u]
        want = mu_base[c, v, u]
        if k > 0:
            for ci, ky, kx in itertools.product(range(C), range(3), range(3)):
                yy, xx = v + ky - 1, u + kx - 1
                if 0 <= yy < h and 0 <= xx < w and part[ci, yy, xx] < k:
                    want += float(wts[f"m{k}"][c, ci, ky, kx]) * r[ci, yy, xx]
        assert abs(mu[c, v, u] - want) < 1e-12


def test_zero_step_weights_reduce_to_single_pass():
    C, h, w = 8, 4, 4
    rng = np.random.default_rng(5)
    wts = {f"m{k}": np.zeros((C, C, 3, 3), np.float32) for k in (1, 2, 3)}
    y = rng.standard_normal((C, h, w)) * 4
    mu_base = rng.standard_normal((C, h, w))
    mu, r = quadtree.encode_means(y, mu_base, wts)
    np.testing.assert_array_equal(mu, mu_base)
    np.testing.assert_array_equal(r, np.clip(np.rint(y - mu_base), -32, 32))


def test_encoder_and_decoder_means_agree():
    C, h, w = 16, 6, 8
    rng = np.random.default_rng(6)
    wts = _weights(C, 7)
    y = rng.standard_normal((C, h, w)) * 5
    mu_base = rng.standard_normal((C, h, w))
    mu_e, r = quadtree.encode_means(y, mu_base, wts)
    mu_d = quadtree.decode_means(r, mu_base, wts)
    np.testing.assert_array_equal(mu_e, mu_d)
    # each residual is the rounding of y minus its own (refined) mean
    np.testing.assert_array_equal(r, np.clip(np.rint(y - mu_e), -32, 32))
    assert np.abs(y - (r + mu_e)).max() <= 0.5 + 1e-12


def test_quadtree_chunk_round_trip_and_flag():
    T, H, W, C = 4, 64, 64, 64
    fr = video_chunk(T, H, W, 3, seed=1)
    wts = stand_in_weights(T, C, quadtree=True)
    base = stand_in_weights(T, C)
    for k in base:   # the base layers' draws are unchanged
        np.testing.assert_array_equal(base[k], wts[k])
    bs, inter = codec.encode_chunk(fr, wts, seg_log2=10, seg_log2_z=8)
    assert container.parse(bs)["flags"] == container.FLAG_QUADTREE
    hdr, dec = codec.decode_latent(bs, wts)
    np.testing.assert_array_equal(dec["y_sym"], inter["y_sym"])
    mu_e, _ = quadtree.encode_means(inter["y"], nets.params(inter["z_hat"], wts, 8, 8)[0], wts)
    np.testing.assert_allclose(dec["y_hat"], codec.from_hwc(inter["y_sym"], C, 8, 8) - 32.0 + mu_e,
                               rtol=0, atol=1e-12)
    # a single-pass model refuses a quadtree stream, and the other way round
    with pytest.raises(container.BadContainer):
        codec.decode_latent(bs, base)
    bs0, _ = codec.encode_chunk(fr, base, seg_log2=10, seg_log2_z=8)
    with pytest.raises(container.BadContainer):
        codec.decode_latent(bs0, wts)
