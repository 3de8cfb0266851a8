"""Entropy model pieces: scale table, index thresholds, symbols, CDF tables.

Test infrastructure only (see the package docstring).

Sec. 3.4: the residual r_hat = round(y - mu) is arithmetic-coded under a
Gaussian of scale sigma, and the decoder recovers r_hat from sigma alone and
adds mu afterwards (y_hat = r_hat + mu).  The paper gives no table sizes; the
readings used here are:

  * 64 scales s_k, log-spaced with both ends inclusive in [0.11, 64];
  * sigma maps to the index of the nearest s_k in the log domain, realised as
    comparisons against float32 geometric midpoints t_j = fl32(sqrt(s_j s_{j+1}))
    (ties go up), so the index needs no transcendental function;
  * 65 symbols r in [-32, 32]; the two edge symbols absorb the Gaussian tails;
  * probabilities are quantised to a 16-bit total: f = 1 + floor(p (M - 65)),
    the deficit goes to the centre symbol, every frequency is at least 1 and
    the table is exactly symmetric.

Pins: thresholds and index at the closed-form special cases (sigma = s_k,
table ends, monotonicity); tables against scipy's normal CDF (|f - M p| is
bounded by the number of symbols) and the invariants sum f = M, f >= 1,
symmetry, strictly increasing cumulative counts, centre mass non-increasing in
the scale.
"""
from __future__ import annotations

import math

import numpy as np

N_SCALES = 64
N_SYMBOLS = 65
PREC = 16
M = 1 << PREC
SIGMA_MIN = 0.11
SIGMA_MAX = 64.0
K_Z = 22  # table row used for every hyper-latent symbol (sigma ~ 1.0)


def scales() -> np.ndarray:
    """s_k = exp(ln 0.11 + k (ln 64 - ln 0.11) / 63), k = 0..63, float64."""
    lo, hi = math.log(SIGMA_MIN), math.log(SIGMA_MAX)
    return np.array([math.exp(lo + k * (hi - lo) / (N_SCALES - 1)) for k in range(N_SCALES)])


def thresholds() -> np.ndarray:
    """t_j = fl32(sqrt(s_j * s_{j+1})), j = 0..62, returned as float32."""
    s = scales()
    return np.array([math.sqrt(s[j] * s[j + 1]) for j in range(N_SCALES - 1)]).astype(np.float32)


def scale_index(sigma: np.ndarray) -> np.ndarray:
    """idx = #{j : sigma >= t_j} in [0, 63]; sigma compared exactly with t_j."""
    t = thresholds().astype(np.float64)
    sig = np.asarray(sigma, dtype=np.float64)
    return (sig[..., None] >= t).sum(axis=-1).astype(np.uint8)


def symbolise(y: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """r_hat = clamp(rint(y - mu), -32, 32), returned as symbol r_hat + 32 (uint8)."""
    r = np.clip(np.rint(np.asarray(y, np.float64) - np.asarray(mu, np.float64)), -32, 32)
    return (r + 32).astype(np.uint8)


def _phi(x: float) -> float:
    """Standard normal CDF via the complementary error function."""
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def gaussian_pmf(s: float) -> np.ndarray:
    """Probabilities of the 65 residual values r = -32..32 under N(0, s^2).

    Integer r takes the mass of [r - 1/2, r + 1/2); r = -32 also takes the
    left tail.  Only r <= 0 is evaluated and mirrored, so the result is
    exactly symmetric.
    """
    p = np.zeros(N_SYMBOLS)
    for r in range(-32, 1):
        if r == 0:
            val = math.erf(0.5 / (s * math.sqrt(2.0)))
        elif r == -32:
            val = _phi((r + 0.5) / s)
        else:
            val = _phi((r + 0.5) / s) - _phi((r - 0.5) / s)
        p[r + 32] = val
        p[32 - r] = val
    return p


def cdf_tables() -> tuple[np.ndarray, np.ndarray]:
    """Quantised frequency and cumulative tables, each (64, 65) uint16-valued.

    Returned as int64 arrays: freq[k, s] and cum[k, s] = sum_{s' < s} freq[k, s'].
    """
    freq = np.zeros((N_SCALES, N_SYMBOLS), dtype=np.int64)
    for k, s in enumerate(scales()):
        p = gaussian_pmf(float(s))
        f = 1 + np.floor(p * (M - N_SYMBOLS)).astype(np.int64)
        f[32] += M - int(f.sum())
        freq[k] = f
    cum = np.zeros_like(freq)
    cum[:, 1:] = np.cumsum(freq, axis=1)[:, :-1]
    return freq, cum


def ideal_bits(sym: np.ndarray, idx: np.ndarray, freq: np.ndarray) -> float:
    """sum of -log2(f_s / M) over coded symbols (the code length target)."""
    f = freq[np.asarray(idx, np.int64), np.asarray(sym, np.int64)].astype(np.float64)
    return float(np.sum(PREC - np.log2(f)))
