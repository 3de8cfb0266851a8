"""Scale index from the log spacing of the thresholds.

The GPU epilogue counts the thresholds <= sigma (the CDF table index) without
a search: the thresholds are float32 geometric midpoints of log-spaced
scales, so 1 + floor((log sigma - log t0) / step), step = log(t62 / t0) / 62,
is within one of the count, and one exact comparison each way against the
float32 table gives it.  These tests pin that premise on the oracle's
thresholds, with the logarithm perturbed by more than a hardware log's error.
"""
import numpy as np
import pytest

from oracle import entropy


def _guess_and_fix(sig, t, lt0, inv_step, pert):
    lg = np.log(sig).astype(np.float32) + np.float32(pert)
    k0 = np.clip(np.floor((lg - lt0) * inv_step).astype(np.int64) + 1, 0, 63)
    lo = np.where(k0 > 0, t[np.maximum(k0 - 1, 0)], -np.inf)
    hi = t[k0]
    return k0, k0 - (lo > sig) + (hi <= sig)


@pytest.mark.parametrize("pert", [-3e-6, 0.0, 3e-6])
def test_log_guess_is_within_one_and_the_fix_is_exact(pert):
    thr = entropy.thresholds().astype(np.float32)
    t = np.concatenate([thr, [np.float32(np.inf)]]).astype(np.float32)
    lt0 = np.float32(np.log(t[0]))
    inv_step = np.float32(62.0) / (np.float32(np.log(t[62])) - lt0)
    rng = np.random.default_rng(3)
    sig = np.exp(rng.uniform(np.log(0.11), np.log(64.0), 1_000_000)).astype(np.float32)
    edge = np.concatenate([np.nextafter(t[:63], np.float32(0)), t[:63],
                           np.nextafter(t[:63], np.float32(np.inf)), [0.11, 64.0]]).astype(np.float32)
    sig = np.clip(np.concatenate([sig, edge]), np.float32(0.11), np.float32(64.0)).astype(np.float32)
    exact = np.searchsorted(t[:63], sig, side="right")
    k0, k = _guess_and_fix(sig, t, lt0, inv_step, pert)
    assert np.abs(k0 - exact).max() <= 1
    np.testing.assert_array_equal(k, exact)
    # the index spans the table: 0 below the first threshold, 63 past the last
    assert exact.min() == 0 and exact.max() == 63
