"""Pins of the rectification oracle (Section 3.2.3, bilinear resampling of
the sensed image into reference geometry): the identity and integer
translations reproduce pixels exactly, half-pixel shifts give neighbour
means, bilinear interpolation reproduces affine intensity ramps exactly at
any position, a scale map samples known pixels, and points outside the
image or behind the projective horizon get the fill value."""
import numpy as np
import pytest

from oracle import rectify_oracle as X


def _img(seed, H, W):
    return np.random.default_rng(seed).uniform(-1, 1, (H, W))


def test_identity_is_exact():
    a = _img(0, 37, 53)
    out = X.rectify(a, np.eye(3), 37, 53, fill=np.nan)
    np.testing.assert_array_equal(out, a)


@pytest.mark.parametrize("dy,dx", [(3, -5), (-7, 2), (0, 11)])
def test_integer_translation_is_a_shifted_copy(dy, dx):
    a = _img(1, 40, 50)
    M = np.array([[1, 0, dy], [0, 1, dx], [0, 0, 1.0]])       # sensed p -> reference p + d
    out = X.rectify(a, M, 40, 50, fill=np.nan)
    for r in range(40):
        for c in range(50):
            sr, sc = r - dy, c - dx
            if 0 <= sr < 40 and 0 <= sc < 50:
                assert out[r, c] == a[sr, sc]
            else:
                assert np.isnan(out[r, c])


def test_half_pixel_shift_is_the_neighbour_mean():
    a = _img(2, 20, 30)
    M = np.array([[1, 0, 0], [0, 1, -0.5], [0, 0, 1.0]])
    out = X.rectify(a, M, 20, 29, fill=np.nan)
    np.testing.assert_allclose(out, 0.5 * (a[:, :-1] + a[:, 1:]), rtol=0, atol=1e-15)


def test_affine_ramp_is_reproduced_at_any_position():
    """Bilinear interpolation is exact on f(y, x) = a + b y + c x."""
    H, W = 64, 80
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = 0.3 + 0.02 * y - 0.015 * x
    rng = np.random.default_rng(3)
    M = np.array([[1.01, 0.02, 1.7], [-0.015, 0.99, -2.3], [2e-5, -1e-5, 1.0]])
    out = X.rectify(f, M, H, W, fill=np.nan)
    py, px, ok = X.source_points(M, H, W)
    inside = ok & (py >= 0) & (py <= H - 1) & (px >= 0) & (px <= W - 1)
    want = 0.3 + 0.02 * py - 0.015 * px
    assert inside.mean() > 0.8
    np.testing.assert_allclose(out[inside], want[inside], rtol=0, atol=1e-12)
    assert np.isnan(out[~inside]).all()
    del rng


def test_scale_samples_known_pixels():
    a = _img(4, 30, 30)
    M = np.diag([0.5, 0.5, 1.0])        # reference = sensed / 2: output (r, c) reads sensed (2r, 2c)
    out = X.rectify(a, M, 15, 15, fill=np.nan)
    np.testing.assert_array_equal(out, a[::2, ::2])


def test_boundary_and_horizon():
    a = _img(5, 10, 10)
    # last row / column exactly: inside, weight 0 on the missing neighbour
    M = np.array([[1, 0, -0.0], [0, 1, 0.0], [0, 0, 1.0]])
    out = X.rectify(a, M, 10, 10, fill=-7.0)
    assert out[9, 9] == a[9, 9]
    # a projective map whose horizon crosses the output: w <= 0 is fill
    P = np.array([[1, 0, 0], [0, 1, 0], [0, 0.2, 1.0]])      # inverse: w = 1 - 0.2 c, <= 0 from c = 5
    py, px, ok = X.source_points(P, 10, 10)
    out = X.rectify(a, P, 10, 10, fill=-7.0)
    np.testing.assert_array_equal(ok, np.broadcast_to(np.arange(10) < 5, (10, 10)))
    assert (out[:, 5:] == -7.0).all()
    # (2, 2): w = 0.6, p = (10/3, 10/3): weights 2/3, 1/3 on rows 3, 4 and columns 3, 4
    want = (4 * a[3, 3] + 2 * a[3, 4] + 2 * a[4, 3] + a[4, 4]) / 9
    assert out[0, 0] == a[0, 0] and out[2, 2] == pytest.approx(want, abs=1e-14)
