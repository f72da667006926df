"""Pins of the RANSAC oracle (Section 3.2.3) against facts that do not come
from its own code: exact recovery of known maps, barycentric brute force of
every three-point hypothesis, the translation special case against the
median consistency check, the word-to-index map at its exact boundaries,
tie-breaking, degenerate samples and the flag rules."""
import itertools

import numpy as np
import pytest

from oracle import ransac_oracle as R
from oracle import sfoc_oracle as O

SIZE = 2048


def _cps(src, dst, flags=None):
    """CP records whose correspondences are src -> dst (pixels); the integer
    part of the displacement goes to dy/dx, the rest to sub_dy/sub_dx."""
    n = len(src)
    c = np.zeros(n, dtype=O.CP_DTYPE)
    c["sen_row"] = src[:, 0].astype(np.int32)
    c["sen_col"] = src[:, 1].astype(np.int32)
    d = dst - np.stack([c["sen_row"], c["sen_col"]], 1)
    c["dy"] = np.round(d[:, 0]).astype(np.int32)
    c["dx"] = np.round(d[:, 1]).astype(np.int32)
    c["sub_dy"] = (d[:, 0] - c["dy"]).astype(np.float32).astype(np.float64)
    c["sub_dx"] = (d[:, 1] - c["dx"]).astype(np.float32).astype(np.float64)
    if flags is not None:
        c["flags"] = flags
    return c


def _points(rng, n, lo=100, hi=SIZE - 100):
    return rng.integers(lo, hi, (n, 2)).astype(np.float64)


def _apply(P, pts):
    q = np.column_stack([pts, np.ones(len(pts))]) @ P.T
    return q[:, :2] / q[:, 2:3]


def _true_dst(c, prior=None):
    """Reference points of CP records, from their fields."""
    py = 0 if prior is None else prior[:, 0]
    px = 0 if prior is None else prior[:, 1]
    return np.stack([c["sen_row"] + py + c["dy"] + c["sub_dy"], c["sen_col"] + px + c["dx"] + c["sub_dx"]], 1)


def _rot(deg, scale, t, persp=(0.0, 0.0)):
    a = np.deg2rad(deg)
    ctr = SIZE / 2
    P = np.array([[scale * np.cos(a), -scale * np.sin(a), 0], [scale * np.sin(a), scale * np.cos(a), 0], [0, 0, 1.0]])
    C = np.array([[1, 0, ctr], [0, 1, ctr], [0, 0, 1.0]])
    Ci = np.array([[1, 0, -ctr], [0, 1, -ctr], [0, 0, 1.0]])
    T = np.array([[1, 0, t[0]], [0, 1, t[1]], [0, 0, 1.0]])
    K = np.array([[1, 0, 0], [0, 1, 0], [persp[0], persp[1], 1.0]])
    M = T @ C @ K @ P @ Ci
    return M / M[2, 2]


def test_word_to_index_boundaries():
    for n in (1, 3, 7, 400, 65537):
        for i in range(0, n, max(1, n // 50)):
            w = -(-(i << 32) // n)                    # smallest word with w * n >= i * 2^32
            assert R.sample_indices([w], n)[0] == i
            if w > 0:
                assert R.sample_indices([w - 1], n)[0] == i - 1
        assert R.sample_indices([2 ** 32 - 1], n)[0] == n - 1
        assert R.sample_indices([0], n)[0] == 0


@pytest.mark.parametrize("seed", range(5))
def test_minimal_affine_is_exact(seed):
    rng = np.random.default_rng(seed)
    A = np.vstack([rng.normal(0, 1, (2, 3)), [0, 0, 1]])
    src = rng.uniform(-1, 1, (3, 2))
    dst = src @ A[:2, :2].T + A[:2, 2]
    M = R.fit_affine(src, dst)
    np.testing.assert_allclose(M, A, atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_minimal_projective_is_exact_and_reduces_to_affine(seed):
    rng = np.random.default_rng(seed)
    P = np.vstack([rng.normal(0, 1, (2, 3)), [*rng.normal(0, 0.2, 2), 1.0]])
    src = rng.uniform(-1, 1, (4, 2))
    dst = _apply(P, src)
    M = R.fit_projective(src, dst)
    np.testing.assert_allclose(M, P, atol=1e-10)
    A = P.copy()
    A[2, :2] = 0.0
    M = R.fit_projective(src, _apply(A, src))
    np.testing.assert_allclose(M[2, :2], 0.0, atol=1e-12)
    np.testing.assert_allclose(M, A, atol=1e-10)


def test_affine_counts_match_barycentric_brute_force():
    """Every three-point hypothesis over six candidates: the count of points
    whose image under the affine map through the sample lies within the
    threshold, with the map evaluated through barycentric coordinates."""
    rng = np.random.default_rng(3)
    src = _points(rng, 6)
    A = _rot(1.0, 1.01, (5.0, -3.0))
    dst = _apply(A, src)
    dst[4] += (9.0, -4.0)
    dst[5] += (-2.0, 1.2)       # an outlier close to the threshold of some hypotheses
    c = _cps(src, dst)
    dst = _true_dst(c)
    n = 6
    subsets = list(itertools.combinations(range(n), 3))
    words = np.array([[-(-(i << 32) // n) for i in s] for s in subsets], dtype=np.uint64).astype(np.uint32)
    _, res = R.ransac(c, words.ravel(), R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    for h, s in enumerate(subsets):
        T = src[list(s)]
        B = np.column_stack([T, np.ones(3)]).T                    # columns: the triangle's vertices
        lam = np.linalg.solve(B, np.column_stack([src, np.ones(n)]).T)   # barycentric coordinates of every point
        img = lam.T @ dst[list(s)]
        want = int(np.sum(np.hypot(*(img - dst).T) <= 1.5))
        assert res["counts"][h] == want, (s, res["counts"][h], want)
    assert res["best"] == int(np.argmax(res["counts"]))


def test_translation_case_matches_median_consistency():
    """Pure translation with a minority of outliers far away: the affine
    RANSAC inliers are exactly the CPs within 1.5 px of the shift, which is
    also what the median-translation check keeps."""
    rng = np.random.default_rng(4)
    src = _points(rng, 120)
    t = np.array([7.25, -3.5])
    dst = src + t + rng.uniform(-0.4, 0.4, src.shape)
    bad = rng.random(120) < 0.3
    dst[bad] += rng.uniform(5, 40, (bad.sum(), 2)) * rng.choice([-1, 1], (bad.sum(), 2))
    c = _cps(src, dst)
    words = np.random.default_rng(5).integers(0, 2 ** 32, 3 * 500, dtype=np.uint64).astype(np.uint32)
    out, res = R.ransac(c, words, R.AFFINE, 1.5, 2, SIZE, SIZE, SIZE, SIZE)
    np.testing.assert_array_equal(res["inliers"], ~bad)
    np.testing.assert_allclose(res["model_px"][:2, :2], np.eye(2), atol=2e-3)
    np.testing.assert_allclose(res["model_px"][:2, 2], t, atol=0.1)
    cons = O.consistency(c.copy())
    np.testing.assert_array_equal(out["flags"], cons["flags"])


@pytest.mark.parametrize("model", [R.AFFINE, R.PROJECTIVE])
def test_recovers_known_model_with_outliers(model):
    rng = np.random.default_rng(6)
    P = _rot(2.0, 1.015, (12.0, -9.0), (3e-6, -2e-6) if model == R.PROJECTIVE else (0.0, 0.0))
    src = _points(rng, 300)
    dst = _apply(P, src)
    bad = rng.random(300) < 0.4
    dst[bad] += rng.uniform(6, 60, (bad.sum(), 2)) * rng.choice([-1, 1], (bad.sum(), 2))
    c = _cps(src, dst)
    k = R.SAMPLE[model]
    words = np.random.default_rng(7).integers(0, 2 ** 32, k * 2000, dtype=np.uint64).astype(np.uint32)
    out, res = R.ransac(c, words, model, 1.5, 2, SIZE, SIZE, SIZE, SIZE)
    np.testing.assert_array_equal(res["inliers"], ~bad)
    # float32 sub-pixel parts carry about 1e-5 px of rounding
    grid = np.stack(np.meshgrid(np.linspace(0, SIZE, 9), np.linspace(0, SIZE, 9)), -1).reshape(-1, 2)
    assert np.abs(_apply(res["model_px"], grid) - _apply(P, grid)).max() < 1e-3
    assert (out["flags"][~bad] == O.VALID).all() and (out["flags"][bad] == O.INCONSISTENT).all()


def test_lowest_index_wins_ties():
    rng = np.random.default_rng(8)
    src = _points(rng, 8)
    dst = src + (3.0, 4.0)
    c = _cps(src, dst)
    n = 8
    w = lambda i: -(-(i << 32) // n)
    a = [w(0), w(1), w(2)]
    b = [w(3), w(5), w(6)]
    _, r1 = R.ransac(c, np.array(a + b, np.uint64).astype(np.uint32), R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    _, r2 = R.ransac(c, np.array(b + a, np.uint64).astype(np.uint32), R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    assert list(r1["counts"]) == [8, 8] and r1["best"] == 0 and r2["best"] == 0
    np.testing.assert_array_equal(r1["model"], r1["models"][0])
    np.testing.assert_array_equal(r2["model"], r2["models"][0])


def test_degenerate_samples_and_no_model():
    rng = np.random.default_rng(9)
    src = np.array([[100, 100], [200, 200], [300, 300], [400, 150], [500, 900]], np.float64)
    dst = src + 2.0
    c = _cps(src, dst)
    n = 5
    w = lambda i: -(-(i << 32) // n)
    words = np.array([w(0), w(1), w(2),        # collinear in both images
                      w(3), w(3), w(4),        # repeated index
                      w(0), w(3), w(4)], np.uint64).astype(np.uint32)
    _, res = R.ransac(c, words, R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    assert list(res["counts"][:2]) == [-1, -1] and res["counts"][2] == 5 and res["best"] == 2
    # every hypothesis degenerate: no model, every eligible CP INCONSISTENT
    out, res = R.ransac(c, words[:6], R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    assert res["model"] is None and (out["flags"] == O.INCONSISTENT).all()
    # fewer candidates than a sample
    out, res = R.ransac(c[:3], words[:4], R.PROJECTIVE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    assert res["model"] is None and list(res["counts"]) == [-1] and (out["flags"] == O.INCONSISTENT).all()
    # nothing eligible: nothing changes
    d = c.copy()
    d["flags"] = O.EDGE_PEAK
    out, res = R.ransac(d, words[:3], R.AFFINE, 1.5, 0, SIZE, SIZE, SIZE, SIZE)
    assert res["n_cand"] == 0 and (out["flags"] == O.EDGE_PEAK).all()
    del rng


def test_flag_rules_and_prior():
    rng = np.random.default_rng(10)
    src = _points(rng, 40)
    prior = rng.integers(-5, 6, (40, 2)).astype(np.int32)
    true = src + (4.0, -6.0)
    bad = np.zeros(40, bool)
    bad[::5] = True
    true[bad] += 20.0
    c = _cps(src, true - prior)           # the records hold displacement minus prior
    flags = np.zeros(40, np.uint32)
    flags[1] = O.OOB
    flags[2] = O.VALID | O.LEARNED
    flags[3] = O.INCONSISTENT
    flags[7] = O.EDGE_PEAK
    c["flags"] = flags
    words = np.random.default_rng(11).integers(0, 2 ** 32, 3 * 300, dtype=np.uint64).astype(np.uint32)
    out, res = R.ransac(c, words, R.AFFINE, 1.5, 1, SIZE, SIZE, SIZE, SIZE, prior=prior)
    assert out["flags"][1] == O.OOB and out["flags"][7] == O.EDGE_PEAK
    assert out["flags"][2] == O.VALID | O.LEARNED
    assert out["flags"][3] == O.VALID
    elig = np.ones(40, bool)
    elig[[1, 7]] = False
    want = np.where(bad, O.INCONSISTENT, O.VALID)
    np.testing.assert_array_equal(out["flags"][elig] & (O.VALID | O.INCONSISTENT), want[elig])
    np.testing.assert_allclose(res["model_px"][:2, 2], (4.0, -6.0), atol=1e-4)


def test_pixel_model_maps_pixels():
    rng = np.random.default_rng(12)
    P = _rot(-1.5, 0.99, (3.0, 2.0), (1e-6, 2e-6))
    src = _points(rng, 50, 50, 700)
    dst = _apply(P, src)
    c = _cps(src, dst)
    words = np.random.default_rng(13).integers(0, 2 ** 32, 4 * 200, dtype=np.uint64).astype(np.uint32)
    _, res = R.ransac(c, words, R.PROJECTIVE, 1.5, 2, 800, 760, 900, 820)
    assert res["inliers"].all()
    np.testing.assert_allclose(_apply(res["model_px"], src), _true_dst(c), atol=1e-4)
