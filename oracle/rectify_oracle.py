"""Plain FP64 CPU reference for image rectification (Section 3.2.3: once the
mismatched CPs are removed, the sensed image is resampled into the
reference image's coordinate system with bilinear interpolation).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call this module.  The GPU
library never uses it and shares no code with it.

Readings (the paper names the step and the interpolation only):
  * The model maps sensed (row, col, 1) to reference coordinates (the model
    RANSAC returns).  Output pixel (r, c) of the rectified image, in the
    reference grid, takes the sensed image at p = model^-1 (r, c, 1),
    dehomogenised.
  * Bilinear interpolation between the four pixels around p with weights
    from its fractional part; p must lie in [0, H-1] x [0, W-1] (an index
    past the last row or column only ever gets weight 0); points outside,
    or whose homogeneous coordinate is <= 0, get the fill value.
"""
from __future__ import annotations

import numpy as np


def source_points(model: np.ndarray, Ho: int, Wo: int):
    """Sensed-image (row, col) of every output pixel, and the mask of
    points with a positive homogeneous coordinate."""
    Minv = np.linalg.inv(np.asarray(model, np.float64))
    r, c = np.meshgrid(np.arange(Ho, dtype=np.float64), np.arange(Wo, dtype=np.float64), indexing="ij")
    P = np.stack([r, c, np.ones_like(r)], -1) @ Minv.T
    w = P[..., 2]
    ok = w > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        py = np.where(ok, P[..., 0] / w, -1.0)
        px = np.where(ok, P[..., 1] / w, -1.0)
    return py, px, ok


def bilinear(img: np.ndarray, py: np.ndarray, px: np.ndarray, fill: float) -> np.ndarray:
    """Bilinear samples of img at (py, px); fill outside [0, H-1] x [0, W-1]."""
    H, W = img.shape
    src = np.asarray(img, np.float64)
    inside = (py >= 0) & (py <= H - 1) & (px >= 0) & (px <= W - 1)
    y0 = np.clip(np.floor(py), 0, H - 1).astype(np.int64)
    x0 = np.clip(np.floor(px), 0, W - 1).astype(np.int64)
    fy = np.where(inside, py - y0, 0.0)
    fx = np.where(inside, px - x0, 0.0)
    y1 = np.minimum(y0 + 1, H - 1)
    x1 = np.minimum(x0 + 1, W - 1)
    v = ((1 - fy) * ((1 - fx) * src[y0, x0] + fx * src[y0, x1]) +
         fy * ((1 - fx) * src[y1, x0] + fx * src[y1, x1]))
    return np.where(inside, v, fill)


def rectify(sen: np.ndarray, model: np.ndarray, Ho: int, Wo: int, fill: float = 0.0) -> np.ndarray:
    """Rectified sensed image in the Ho x Wo reference grid (float64)."""
    py, px, ok = source_points(model, Ho, Wo)
    out = bilinear(sen, py, px, fill)
    return np.where(ok, out, fill)
