"""Quadtree partition of the latent and four-step progressive means.

Test infrastructure only (see the package docstring).

Sec. 3.4 with the Fig. 3 caption (a): the quantised latent is split into four
partitions in the quadtree manner of DCVC-DC.  The streamlined model predicts
the scales of *all four* partitions and the mean of the first in one pass
from the prior; the bit-stream is read in one step using the scales alone;
the means of partitions 1, 2 and 3 are then estimated one after another, each
from the partitions decoded before it, entirely on the GPU.

The figure itself is missing from the text, so the geometry is a reading:

  * channel group g = floor(4 c / C) (C divisible by 4) and spatial phase
    q = 2 (v mod 2) + (u mod 2) of element (c, v, u);
  * group 0 takes its phases in the order TL, BR, TR, BL (q = 0, 3, 1, 2):
    rank(q) = 0, 2, 3, 1 for q = 0, 1, 2, 3;
  * partition(c, v, u) = (rank(q) + g) mod 4.

Every partition then holds one channel group of every position and one
spatial phase of every channel group (a Latin square over group x phase),
so each step mixes spatial and channel context.

Mean estimation, one step per partition k = 1, 2, 3 (a reading too: the paper
gives no network internals):

  delta_k = conv3x3(M_<k * r_hat, Wm_k)            (C -> C, no bias)
  mu[part k] = mu_base[part k] + delta_k[part k]

mu_base is the single pass's mean (the prior's estimate for every element;
partition 0 keeps it), M_<k the indicator of partitions 0..k-1 and r_hat the
decoded residual symbols of those partitions.  The step input is r_hat rather
than y_hat = r_hat + mu: given the prior, both carry the same information,
and integer inputs keep every product exact on the GPU, so encoder and
decoder derive bit-identical means.  The encoder quantises partition k with
its refined mean, r_hat = clamp(rint(y - mu), -32, 32), before step k + 1.

Pins: the partition's counting and Latin-square properties; causality (the
mean of partition k does not move when any element of partitions >= k
changes); a brute-force per-element sum over the causal neighbourhood; zero
step weights reduce to the single pass; decoder means equal encoder means.
The geometry against the paper's figure is parity unpinned (no figure).
"""
from __future__ import annotations

import numpy as np

from . import nets

# rank of spatial phase q = 2 (v mod 2) + (u mod 2) for channel group 0
PHASE_RANK = (0, 2, 3, 1)
N_PARTS = 4


def partition(C: int, h: int, w: int) -> np.ndarray:
    """Partition index (0..3) of every latent element, shape (C, h, w)."""
    if C % N_PARTS:
        raise ValueError("C must be divisible by 4")
    g = (N_PARTS * np.arange(C)) // C
    v = np.arange(h)
    u = np.arange(w)
    q = 2 * (v[:, None] % 2) + (u[None, :] % 2)
    rank = np.asarray(PHASE_RANK)[q]
    return (rank[None, :, :] + g[:, None, None]) % N_PARTS


def _step_delta(r_hat: np.ndarray, part: np.ndarray, k: int, wts: dict) -> np.ndarray:
    """conv3x3 of the residuals of partitions 0..k-1 (others zero) with Wm_k."""
    return nets.conv(np.where(part < k, r_hat, 0.0), wts[f"m{k}"])


def encode_means(y: np.ndarray, mu_base: np.ndarray, wts: dict):
    """Encoder side: returns (mu, r_hat), both (C, h, w) float64.

    Partition 0 is quantised with mu_base; partition k = 1..3 with
    mu_base + delta_k, where delta_k sees only the residuals already fixed.
    """
    C, h, w = y.shape
    part = partition(C, h, w)
    mu = np.array(mu_base, dtype=np.float64)
    r_hat = np.zeros_like(mu)
    sel = part == 0
    r_hat[sel] = nets.rint_clamp(y[sel] - mu[sel])
    for k in range(1, N_PARTS):
        d = _step_delta(r_hat, part, k, wts)
        sel = part == k
        mu[sel] = mu_base[sel] + d[sel]
        r_hat[sel] = nets.rint_clamp(y[sel] - mu[sel])
    return mu, r_hat


def decode_means(r_hat: np.ndarray, mu_base: np.ndarray, wts: dict) -> np.ndarray:
    """Decoder side: every r_hat is already decoded (one bit-stream step);
    the means of partitions 1..3 follow one after another.  Returns mu."""
    C, h, w = r_hat.shape
    part = partition(C, h, w)
    mu = np.array(mu_base, dtype=np.float64)
    for k in range(1, N_PARTS):
        d = _step_delta(r_hat, part, k, wts)
        sel = part == k
        mu[sel] = mu_base[sel] + d[sel]
    return mu
