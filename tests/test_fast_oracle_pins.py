"""Pins of the block-based FAST oracle (Section 3.1.1; FAST as Rosten and
Drummond define it): the corner strength against the segment test itself,
contrast and rotation symmetries, uniform images and straight edges, the
corners of a blurred square, the suppression tie rule, and the per-block
selection against repeated arg-max picking."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import fast_oracle as F


def _structured(seed, H, W):
    rng = np.random.default_rng(seed)
    a = ndimage.gaussian_filter(rng.uniform(0, 1, (H, W)), 1.2)
    for _ in range(6):
        y0, x0 = rng.integers(0, H - 10), rng.integers(0, W - 10)
        a[y0:y0 + rng.integers(5, 15), x0:x0 + rng.integers(5, 15)] += rng.uniform(-0.5, 0.5)
    return a.astype(np.float32)


def test_strength_is_the_largest_passing_threshold():
    a = _structured(0, 48, 56)
    V = F.strength(a, 3)
    checked = 0
    for y in range(3, 45):
        for x in range(3, 53):
            v = V[y, x]
            if v <= 0:
                continue
            assert not F.segment_test(a, y, x, float(v))                        # fails at V
            assert F.segment_test(a, y, x, float(np.nextafter(v, np.float32(-np.inf))))   # passes just below
            checked += 1
    assert checked > 100


def test_contrast_inversion_and_rotation():
    a = _structured(1, 40, 40)
    V = F.strength(a, 3)
    np.testing.assert_array_equal(F.strength(-a, 3), V)
    np.testing.assert_array_equal(F.strength(np.ascontiguousarray(np.rot90(a)), 3), np.rot90(V))
    np.testing.assert_array_equal(F.strength(np.ascontiguousarray(a.T), 3), V.T)


def test_uniform_and_straight_edges_are_not_corners():
    assert (F.strength(np.full((20, 20), 0.7, np.float32), 3)[3:-3, 3:-3] == 0).all()
    y, x = np.mgrid[0:30, 0:30].astype(np.float32)
    for ramp in (0.1 * x, 0.05 * y, 0.03 * x + 0.07 * y):
        assert (F.strength(ramp, 3)[3:-3, 3:-3] <= 1e-6).all()
    step = (x >= 15).astype(np.float32)
    assert (F.strength(step, 3)[3:-3, 3:-3] <= 0).all()        # a straight step edge: at most 8 of 16 differ


def test_corners_of_a_blurred_square():
    a = np.zeros((64, 64), np.float32)
    a[20:44, 16:40] = 1.0
    a = ndimage.gaussian_filter(a, 1.0).astype(np.float32)
    ips, sc, cnt = F.detect(a, 0.1, 3, 1, 1, 50)
    corners = np.array([[20, 16], [20, 39], [43, 16], [43, 39]])
    d = np.abs(ips[:, None, :] - corners[None]).max(-1)
    assert len(ips) == 4
    assert (d.min(1) <= 2).all() and (d.min(0) <= 2).all()


def test_suppression_tie_rule():
    V = np.full((7, 7), -np.inf, np.float32)
    V[2:4, 2:4] = 5.0                 # a 2x2 plateau: only its raster-first pixel is kept
    V[5, 5] = 3.0
    V[5, 4] = 3.0                     # two equal neighbours in a row: the left one
    keep = F.suppress(V, 1.0)
    assert sorted(zip(*np.nonzero(keep))) == [(2, 2), (5, 4)]


@pytest.mark.parametrize("nby,nbx,per", [(1, 1, 5), (3, 4, 2), (5, 2, 7)])
def test_block_selection_by_repeated_argmax(nby, nbx, per):
    a = _structured(2, 90, 77)
    b = 6
    ips, sc, cnt = F.detect(a, 0.02, b, nby, nbx, per)
    keep = F.suppress(F.strength(a, b), 0.02)
    V = F.strength(a, b)
    H, W = a.shape
    ys = [b + i * (H - 2 * b) // nby for i in range(nby + 1)]
    xs = [b + j * (W - 2 * b) // nbx for j in range(nbx + 1)]
    assert ys[0] == b and ys[-1] == H - b and xs[-1] == W - b
    k = 0
    for i in range(nby):
        for j in range(nbx):
            cand = {(y, x): V[y, x] for y in range(ys[i], ys[i + 1]) for x in range(xs[j], xs[j + 1]) if keep[y, x]}
            picked = []
            while cand and len(picked) < per:
                best = max(cand.items(), key=lambda kv: (kv[1], -(kv[0][0] * W + kv[0][1])))
                picked.append(best[0])
                del cand[best[0]]
            assert cnt[i * nbx + j] == len(picked)
            for q in picked:
                assert tuple(ips[k]) == q and sc[k] == V[q]
                k += 1
    assert k == len(ips)
    assert (ips[:, 0] >= b).all() and (ips[:, 0] < H - b).all() and (ips[:, 1] >= b).all()
