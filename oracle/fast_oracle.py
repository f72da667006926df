"""Plain CPU reference for block-based FAST interest-point detection
(Section 3.1.1: the FAST operator of Rosten and Drummond applied with a
partitioning strategy, so that the interest points are spread evenly over
the image).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call this module.  The GPU
library never uses it and shares no code with it.

The paper names the operator and the partitioning only.  Readings (each
listed with its justification in the design notes):
  * Segment test FAST-9 on the 16-pixel Bresenham circle of radius 3: p is
    a corner for threshold t when 9 cyclically contiguous circle pixels are
    all brighter than I_p + t or all darker than I_p - t.
  * Corner strength V(p) = the largest threshold at which the test still
    passes, i.e. the maximum over the 16 arcs of 9 of
    max(min over the arc of (I_x - I_p), min over the arc of (I_p - I_x));
    p is a corner when V(p) > t.  V decides which pixels become interest
    points, so it is computed in float32, the precision of the image and
    of the kernels: the differences are float32 subtractions and the rest
    is min / max, all exact operations on both sides.
  * Only pixels at least b = max(3, margin) from every border are tested
    (the detection region).
  * Non-maximum suppression over the 3x3 neighbourhood inside the region:
    a corner is kept when its V is greater than that of every neighbour
    before it in raster order and not less than that of every neighbour
    after it.
  * Blocks: the region split into nby x nbx blocks at integer boundaries
    b + floor(i * Hd / nby) (Hd = H - 2b), likewise for columns; in each
    block the per_block kept corners of largest V, ties to the smaller
    raster index.  Output in block order (row-major), within a block by
    rank.
"""
from __future__ import annotations

import numpy as np

# The FAST circle, clockwise from the top: (dy, dx).
CIRCLE = [(-3, 0), (-3, 1), (-2, 2), (-1, 3), (0, 3), (1, 3), (2, 2), (3, 1),
          (3, 0), (3, -1), (2, -2), (1, -3), (0, -3), (-1, -3), (-2, -2), (-3, -1)]
ARC = 9


def strength(img: np.ndarray, b: int) -> np.ndarray:
    """V over the whole image in float32; -inf outside the detection
    region (rows and columns [b, size - b))."""
    a = np.asarray(img, np.float32)
    H, W = a.shape
    V = np.full((H, W), -np.inf, np.float32)
    if H - 2 * b <= 0 or W - 2 * b <= 0:
        return V
    c = a[b:H - b, b:W - b]
    ring = np.stack([a[b + dy:H - b + dy, b + dx:W - b + dx] for dy, dx in CIRCLE])   # (16, h, w)
    up = ring - c[None]          # float32: I_x - I_p
    dn = c[None] - ring          # float32: I_p - I_x
    best = np.full(c.shape, -np.inf, np.float32)
    for k in range(16):
        idx = [(k + j) % 16 for j in range(ARC)]
        best = np.maximum(best, np.maximum(up[idx].min(0), dn[idx].min(0)))
    V[b:H - b, b:W - b] = best
    return V


def segment_test(img: np.ndarray, y: int, x: int, t: float) -> bool:
    """The FAST-9 segment test at (y, x) for threshold t, as a count of
    contiguous circle pixels (float32 comparisons)."""
    a = np.asarray(img, np.float32)
    p = a[y, x]
    ring = [a[y + dy, x + dx] for dy, dx in CIRCLE]
    for sign in (1, -1):
        flags = [(np.float32(sign) * (v - p)) > np.float32(t) for v in ring]
        run = 0
        for f in flags + flags:
            run = run + 1 if f else 0
            if run >= ARC:
                return True
    return False


def suppress(V: np.ndarray, t: float) -> np.ndarray:
    """Kept corners: V > t and the raster-order 3x3 maximum rule."""
    H, W = V.shape
    P = np.full((H + 2, W + 2), -np.inf, np.float32)
    P[1:-1, 1:-1] = V
    keep = V > np.float32(t)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            N = P[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx]
            before = dy < 0 or (dy == 0 and dx < 0)
            keep &= (V > N) if before else (V >= N)
    return keep


def block_bounds(lo: int, n: int, nb: int):
    return [lo + (i * n) // nb for i in range(nb + 1)]


def detect(img: np.ndarray, threshold: float, margin: int, nby: int, nbx: int, per_block: int):
    """(ips (k, 2) int32 (row, col), scores (k,) float32, counts (nby*nbx,)
    int32) of block-based FAST."""
    a = np.asarray(img, np.float32)
    H, W = a.shape
    b = max(3, margin)
    V = strength(a, b)
    keep = suppress(V, threshold)
    ys = block_bounds(b, max(0, H - 2 * b), nby)
    xs = block_bounds(b, max(0, W - 2 * b), nbx)
    ips, scores, counts = [], [], []
    for i in range(nby):
        for j in range(nbx):
            yy, xx = np.nonzero(keep[ys[i]:ys[i + 1], xs[j]:xs[j + 1]])
            yy = yy + ys[i]
            xx = xx + xs[j]
            v = V[yy, xx]
            order = np.lexsort((yy * W + xx, -v.astype(np.float64)))[:per_block]
            counts.append(len(order))
            for q in order:
                ips.append((yy[q], xx[q]))
                scores.append(v[q])
    return (np.array(ips, np.int32).reshape(-1, 2), np.array(scores, np.float32),
            np.array(counts, np.int32))
