"""Three-part bf16 split of float32 weights (entropy-parameter conv).

The library runs the float32 entropy-parameter conv on bf16 matrix cores by
writing every float32 weight w as h + m + l with h = bf16(w),
m = bf16(w - h), l = bf16(w - h - m).  The premise is that the split is
exact: 3 x 8 significant bits hold w's 24, and the residuals are exact
float32 differences.  (The library re-checks every weight when it loads a
model and refuses the model otherwise.)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synthetic import stand_in_weights  # noqa: E402


def split3(w: np.ndarray):
    t = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32))
    h = t.to(torch.bfloat16).float()
    r1 = t - h
    m = r1.to(torch.bfloat16).float()
    r2 = r1 - m
    lo = r2.to(torch.bfloat16).float()
    return h.numpy(), m.numpy(), lo.numpy(), r2.numpy()


def _check(w):
    h, m, lo, r2 = split3(w)
    assert np.array_equal(lo, r2)  # the last residual is a bf16 value
    total = h.astype(np.float64) + m.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, w.astype(np.float64))


@pytest.mark.parametrize("T,C", [(4, 64), (8, 128), (2, 16)])
def test_stand_in_params_weights_split_exactly(T, C):
    _check(stand_in_weights(T, C)["p"])


def test_float32_values_split_exactly():
    rng = np.random.default_rng(11)
    n = 200_000
    # random significands over exponents -100..100, both signs, plus the
    # values next to powers of two and halfway cases of the first rounding
    mant = rng.uniform(1.0, 2.0, n)
    expo = rng.integers(-100, 101, n)
    w = (np.where(rng.random(n) < 0.5, -1.0, 1.0) * np.ldexp(mant, expo)).astype(np.float32)
    bits = rng.integers(0, 1 << 23, 4096).astype(np.uint32) | np.uint32(0x3F800000)
    edge = np.concatenate([bits, bits | np.uint32(0x8000), (bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000),
                           np.array([0x3F800000, 0x3F7FFFFF, 0x3F808000, 0x3F818000], np.uint32)])
    _check(np.concatenate([w, edge.view(np.float32), -edge.view(np.float32)]))


def test_a_two_part_split_is_not_exact():
    # the third part is needed: h + m alone misses the low bits of most weights
    w = stand_in_weights(4, 64)["p"]
    h, m, _, _ = split3(w)
    assert (h.astype(np.float64) + m.astype(np.float64) != w.astype(np.float64)).mean() > 0.9
