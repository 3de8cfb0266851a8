"""The depth-wise convolution block (DC block), float64.

Test infrastructure only (see the package docstring).

The supplementary material builds every module of the paper's codec from one
primitive, the DC block of DCVC-RT; its structure is given only as a figure,
which is missing from the text.  The reading used here keeps what the name
and the cited lineage fix (a depth-wise 3 x 3 spatial convolution between
point-wise channel mixings, with residual connections, followed by a
point-wise feed-forward stage) and nothing else:

  t  = relu(pw1 x)                 pw1: C -> C, 1 x 1
  d  = dw3x3 t                     one 3 x 3 filter per channel, zero padding
  x1 = x + pw2 d                   pw2: C -> C
  u  = relu(pw3 x1)                pw3: C -> 2C
  y  = x1 + pw4 u                  pw4: 2C -> C

No biases (as everywhere in the stand-in).  Weights: pw1 (C, C), dw (C, 3, 3),
pw2 (C, C), pw3 (2C, C), pw4 (C, 2C), float32 values, (out, in) order.

Pins: the point-wise steps against a brute-force per-element sum; the
depth-wise step against torch's grouped conv2d in float64 and against
oracle.nets.conv with a diagonal weight tensor; the residual structure
(all-zero pw2 and pw4 give the identity); linearity of the point-wise part.
"""
from __future__ import annotations

import numpy as np

from . import nets


def pointwise(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """1 x 1 convolution: out[o, v, u] = sum_i w[o, i] x[i, v, u]."""
    return np.tensordot(np.asarray(w, np.float64), np.asarray(x, np.float64), axes=(1, 0))


def depthwise3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """out[c, v, u] = sum_{ky, kx} w[c, ky, kx] x[c, v + ky - 1, u + kx - 1], zero padding."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    w64 = np.asarray(w, np.float64)
    out = np.zeros((C, H, W))
    for ky in range(3):
        for kx in range(3):
            out += w64[:, ky, kx][:, None, None] * xp[:, ky:ky + H, kx:kx + W]
    return out


def dc_block(x: np.ndarray, wts: dict) -> np.ndarray:
    """One DC block on a (C, h, w) feature map (see the module docstring)."""
    x = np.asarray(x, np.float64)
    t = nets.relu(pointwise(x, wts["pw1"]))
    d = depthwise3x3(t, wts["dw"])
    x1 = x + pointwise(d, wts["pw2"])
    u = nets.relu(pointwise(x1, wts["pw3"]))
    return x1 + pointwise(u, wts["pw4"])
