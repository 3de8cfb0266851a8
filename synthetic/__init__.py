"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only produces *data*: video chunks shaped like the paper's 1080p /
720p / 2160p test material (Sec. 4.1 evaluates on such videos; they are not
available here, so textured, shifting synthetic frames stand in for them) and
the stand-in network's random weights (the paper's trained weights are not
used).  It contains none of the codec's arithmetic: no convolution, no entropy
model, no coding.  Both the oracle and the GPU path consume its output.

Video recipe (one chunk):
  * ``rng = numpy.random.default_rng([seed, chunk_id])``; draws happen in the
    order lattice, shifts, noise.
  * A base canvas of (H + 2S) x (W + 2S) pixels per RGB channel, S = max shift.
    Each channel is an i.i.d. U[0,1) lattice on nodes -1..9 x -1..9 (8 x 8 cells
    plus a support ring) interpolated with the Keys cubic kernel (a = -0.5) at
    lattice coordinates 8 (v + 1/2) / (H + 2S) and 8 (u + 1/2) / (W + 2S).
  * Frame t is the canvas window shifted by an integer (dy, dx) drawn uniformly
    from [-S, S], plus N(0, (2/255)^2) noise, clipped to [0, 1], float32.

Weight recipe: ``rng = numpy.random.default_rng([0, T, C])``; layers drawn in
the order listed by :func:`weight_shapes`, each He-normal
``standard_normal(shape) * sqrt(2 / (Cin * 9))`` rounded to float32, OIHW.
"""
from __future__ import annotations

import numpy as np

__all__ = ["video_chunk", "weight_shapes", "stand_in_weights", "dc_block_weights",
           "feature_map", "Z_CHANNELS"]

# Channels of the hyper latent z in the stand-in network.
Z_CHANNELS = 32


def _keys_cubic(d: np.ndarray, a: float = -0.5) -> np.ndarray:
    """Keys (1981) cubic convolution kernel evaluated at offsets ``d``."""
    d = np.abs(d)
    out = np.zeros_like(d)
    m1 = d <= 1.0
    m2 = (d > 1.0) & (d < 2.0)
    out[m1] = (a + 2.0) * d[m1] ** 3 - (a + 3.0) * d[m1] ** 2 + 1.0
    out[m2] = a * d[m2] ** 3 - 5.0 * a * d[m2] ** 2 + 8.0 * a * d[m2] - 4.0 * a
    return out


def _interp_matrix(n_px: int) -> np.ndarray:
    """(n_px, 11) matrix mapping lattice nodes -1..9 to pixel centres."""
    coord = 8.0 * (np.arange(n_px, dtype=np.float64) + 0.5) / n_px
    nodes = np.arange(-1, 10, dtype=np.float64)
    return _keys_cubic(coord[:, None] - nodes[None, :])


def video_chunk(T: int, H: int, W: int, max_shift: int, seed: int = 1,
                chunk_id: int = 0) -> np.ndarray:
    """Return one chunk of T RGB frames, float32, shape (T, 3, H, W), in [0, 1]."""
    rng = np.random.default_rng([seed, chunk_id])
    S = int(max_shift)
    Hc, Wc = H + 2 * S, W + 2 * S
    lattice = rng.random((3, 11, 11))
    shifts = rng.integers(-S, S + 1, size=(T, 2))
    noise = rng.standard_normal((T, 3, H, W), dtype=np.float32)
    my = _interp_matrix(Hc)
    mx = _interp_matrix(Wc)
    canvas = np.einsum("vi,cij,uj->cvu", my, lattice, mx)
    frames = np.empty((T, 3, H, W), dtype=np.float32)
    for t in range(T):
        dy, dx = int(shifts[t, 0]), int(shifts[t, 1])
        win = canvas[:, S + dy:S + dy + H, S + dx:S + dx + W]
        frames[t] = np.clip(win + noise[t] * (2.0 / 255.0), 0.0, 1.0)
    return frames


def weight_shapes(T: int, C: int, quadtree: bool = False, temporal: bool = False
                  ) -> list[tuple[str, tuple[int, int, int, int]]]:
    """Names and OIHW shapes of the stand-in network's conv layers, in draw order.

    quadtree adds the three mean-step layers m1, m2, m3 (C x C), drawn after
    the frame heads, so the other layers' draws are those of the base model.
    temporal adds, after those, the context network c1, c2 (C x C) and the
    context inputs of a1 (a1c, C x C), of the entropy parameters (pc, 2C x C)
    and of d1 (d1c, C x C).
    """
    shapes = [
        ("a1", (C, 192 * T, 3, 3)),
        ("a2", (C, C, 3, 3)),
        ("a3", (C, C, 3, 3)),
        ("h", (Z_CHANNELS, C, 3, 3)),
        ("p", (2 * C, Z_CHANNELS, 3, 3)),
        ("d1", (C, C, 3, 3)),
        ("d2", (C, C, 3, 3)),
        ("d3", (C, C, 3, 3)),
    ]
    for t in range(T):
        shapes.append((f"k1_{t}", (C, C, 3, 3)))
        shapes.append((f"k2_{t}", (C, C, 3, 3)))
        shapes.append((f"k3_{t}", (192, C, 3, 3)))
    if quadtree:
        shapes += [(f"m{k}", (C, C, 3, 3)) for k in (1, 2, 3)]
    if temporal:
        shapes += [("c1", (C, C, 3, 3)), ("c2", (C, C, 3, 3)), ("a1c", (C, C, 3, 3)),
                   ("pc", (2 * C, C, 3, 3)), ("d1c", (C, C, 3, 3))]
    return shapes


def stand_in_weights(T: int, C: int, quadtree: bool = False, temporal: bool = False
                     ) -> dict[str, np.ndarray]:
    """Seeded He-normal weights for the (T, C) stand-in model, float32 OIHW."""
    rng = np.random.default_rng([0, T, C])
    out: dict[str, np.ndarray] = {}
    for name, shape in weight_shapes(T, C, quadtree, temporal):
        cin = shape[1]
        out[name] = (rng.standard_normal(shape) * np.sqrt(2.0 / (cin * 9))).astype(np.float32)
    return out


def dc_block_weights(C: int, seed: int = 0) -> dict[str, np.ndarray]:
    """Seeded He-normal weights of one DC block (C channels), float32.

    ``rng = numpy.random.default_rng([1, C, seed])``; drawn in the order pw1
    (C, C), dw (C, 3, 3), pw2 (C, C), pw3 (2C, C), pw4 (C, 2C), each
    ``standard_normal(shape) * sqrt(2 / fan_in)`` (fan_in = C, 9, C, C, 2C)
    rounded to float32, (out, in) order.
    """
    rng = np.random.default_rng([1, C, seed])
    shapes = [("pw1", (C, C), C), ("dw", (C, 3, 3), 9), ("pw2", (C, C), C),
              ("pw3", (2 * C, C), C), ("pw4", (C, 2 * C), 2 * C)]
    return {n: (rng.standard_normal(s) * np.sqrt(2.0 / f)).astype(np.float32) for n, s, f in shapes}


def feature_map(C: int, h: int, w: int, seed: int = 0) -> np.ndarray:
    """A seeded (C, h, w) float32 latent-resolution feature map: unit-variance
    Gaussian values (the scale of the stand-in network's activations)."""
    rng = np.random.default_rng([2, C, h, w, seed])
    return rng.standard_normal((C, h, w)).astype(np.float32)
