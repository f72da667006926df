"""Plain FP64 CPU reference for RANSAC outlier rejection over control points
(Section 3.2.3: once matching is done, RANSAC removes mismatched CPs, with a
projective model in general and an affine compensation model in the
RPC-based variant; RANSAC itself is Fischler and Bolles' random sample
consensus).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call this module.  The GPU
library never uses it and shares no code with it.

The paper names the method and the models but fixes none of the numbers.
Readings (each listed with its justification in the design notes):
  * Candidates: CPs with an interior peak (none of OOB, FLAT_T, FLAT_S,
    EDGE_PEAK, NONFINITE), in CP order.  A candidate maps the sensed point
    (row, col) to the reference point (row + prior_y + dy + sub_dy,
    col + prior_x + dx + sub_dx).
  * Coordinates are normalised per image before fitting:
    v_n = (v - (size - 1) / 2) * s_inv with s_inv = 1 / (max(H, W) / 2).
  * Hypothesis h takes its k sample indices (k = 3 affine, 4 projective)
    from k caller-supplied 32-bit random words w: index = floor(w * n / 2^32)
    for n candidates.  A sample with a repeated index, or with three
    collinear points (|cross product| <= 1e-9 in normalised units) in either
    image, is degenerate and scores -1.
  * Minimal fit: the unique affine map through three correspondences, or the
    unique homography with h22 = 1 through four.
  * Inlier: reprojection distance in reference pixels <= threshold (1.5 by
    default, the correctness threshold of Section 4.1).  Under a projective
    model a point whose denominator is <= 0 is an outlier.
  * Selection: most inliers; ties go to the lowest hypothesis index.
  * Refinement: n_refine times, a least-squares fit over the current inliers
    (for the projective model the algebraic one with h22 = 1), then the
    inlier set is recomputed.  Fewer than k inliers or a singular system
    stops the refinement with the current model.
  * Output: eligible inliers VALID, eligible outliers INCONSISTENT (both
    bits cleared first).  With no model (fewer than k candidates, or every
    hypothesis degenerate) every eligible CP is INCONSISTENT.  The model is
    returned in pixel coordinates, 3 x 3 row-major, mapping the sensed
    (row, col, 1) to the reference, scaled so that entry (2, 2) is 1.
"""
from __future__ import annotations

import numpy as np

from oracle.sfoc_oracle import EDGE_PEAK, FLAT_S, FLAT_T, INCONSISTENT, NONFINITE, OOB, VALID

AFFINE, PROJECTIVE = 6, 8          # model ids (= free parameters)
SAMPLE = {AFFINE: 3, PROJECTIVE: 4}
COLLINEAR_EPS = 1e-9
BAD = OOB | FLAT_T | FLAT_S | EDGE_PEAK | NONFINITE


def normaliser(H: int, W: int):
    """(centre_row, centre_col, s_inv) of an H x W image."""
    return 0.5 * (H - 1), 0.5 * (W - 1), 1.0 / (0.5 * max(H, W))


def candidates(cps: np.ndarray, prior=None):
    """Indices of the eligible CPs and their correspondences in pixels:
    src (n, 2) sensed (row, col), dst (n, 2) reference (row, col)."""
    idx = np.nonzero((cps["flags"] & BAD) == 0)[0]
    py = np.zeros(len(cps), np.int64) if prior is None else np.asarray(prior)[:, 0].astype(np.int64)
    px = np.zeros(len(cps), np.int64) if prior is None else np.asarray(prior)[:, 1].astype(np.int64)
    c = cps[idx]
    src = np.stack([c["sen_row"], c["sen_col"]], 1).astype(np.float64)
    ir = (c["sen_row"].astype(np.int64) + py[idx] + c["dy"]).astype(np.float64)
    ic = (c["sen_col"].astype(np.int64) + px[idx] + c["dx"]).astype(np.float64)
    dst = np.stack([ir + c["sub_dy"].astype(np.float64), ic + c["sub_dx"].astype(np.float64)], 1)
    return idx, src, dst


def normalise(pts: np.ndarray, H: int, W: int) -> np.ndarray:
    cr, cc, s = normaliser(H, W)
    return np.stack([(pts[:, 0] - cr) * s, (pts[:, 1] - cc) * s], 1)


def sample_indices(words: np.ndarray, n: int) -> np.ndarray:
    """floor(w * n / 2^32) for each 32-bit word."""
    return ((np.asarray(words, dtype=np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def cross(a, b, c) -> float:
    """Twice the signed area of triangle (a, b, c)."""
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def degenerate(src: np.ndarray, dst: np.ndarray, sel: np.ndarray) -> bool:
    """Repeated index, or three collinear points in either image."""
    if len(set(sel.tolist())) < len(sel):
        return True
    k = len(sel)
    for pts in (src, dst):
        for a in range(k):
            for b in range(a + 1, k):
                for c in range(b + 1, k):
                    if abs(cross(pts[sel[a]], pts[sel[b]], pts[sel[c]])) <= COLLINEAR_EPS:
                        return True
    return False


def fit_affine(src: np.ndarray, dst: np.ndarray):
    """3x3 matrix of the affine map with dst = A [src; 1]: least squares over
    the given correspondences (exact for three)."""
    X = np.column_stack([src, np.ones(len(src))])
    if len(src) == 3:
        try:
            sol = np.linalg.solve(X, dst)
        except np.linalg.LinAlgError:
            return None
    else:
        if np.linalg.matrix_rank(X) < 3:
            return None
        sol = np.linalg.lstsq(X, dst, rcond=None)[0]
    M = np.eye(3)
    M[0, :] = sol[:, 0]
    M[1, :] = sol[:, 1]
    return M


def dlt_rows(src: np.ndarray, dst: np.ndarray):
    """The linear system of a homography with h22 = 1: for each
    correspondence (x, y) -> (u, v): u = (h0 x + h1 y + h2) / (h6 x + h7 y + 1)
    and likewise v, multiplied out."""
    n = len(src)
    A = np.zeros((2 * n, 8))
    b = np.zeros(2 * n)
    x, y = src[:, 0], src[:, 1]
    u, v = dst[:, 0], dst[:, 1]
    A[0::2, 0], A[0::2, 1], A[0::2, 2] = x, y, 1.0
    A[0::2, 6], A[0::2, 7] = -x * u, -y * u
    A[1::2, 3], A[1::2, 4], A[1::2, 5] = x, y, 1.0
    A[1::2, 6], A[1::2, 7] = -x * v, -y * v
    b[0::2], b[1::2] = u, v
    return A, b


def fit_projective(src: np.ndarray, dst: np.ndarray):
    """3x3 homography with h22 = 1: exact through four correspondences,
    algebraic least squares over more."""
    A, b = dlt_rows(src, dst)
    try:
        if len(src) == 4:
            h = np.linalg.solve(A, b)
        else:
            if np.linalg.matrix_rank(A) < 8:
                return None
            h = np.linalg.lstsq(A, b, rcond=None)[0]
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(h)):
        return None
    return np.append(h, 1.0).reshape(3, 3)


def fit(model: int, src, dst):
    return fit_affine(src, dst) if model == AFFINE else fit_projective(src, dst)


def residuals(M: np.ndarray, src: np.ndarray, dst: np.ndarray, s_ref: float) -> np.ndarray:
    """Reprojection distance in reference pixels (normalised coordinates in,
    s_ref = pixels per normalised unit); +inf where the projective
    denominator is <= 0."""
    P = np.column_stack([src, np.ones(len(src))]) @ M.T
    w = P[:, 2]
    out = np.full(len(src), np.inf)
    ok = w > 0
    pr = P[ok, 0] / w[ok]
    pc = P[ok, 1] / w[ok]
    out[ok] = np.hypot((pr - dst[ok, 0]) * s_ref, (pc - dst[ok, 1]) * s_ref)
    return out


def to_pixels(M: np.ndarray, Hs: int, Ws: int, Hr: int, Wr: int) -> np.ndarray:
    """Model in normalised coordinates -> model in pixels."""
    cr, cc, s = normaliser(Hs, Ws)
    Ts = np.array([[s, 0, -cr * s], [0, s, -cc * s], [0, 0, 1.0]])
    cr2, cc2, s2 = normaliser(Hr, Wr)
    Tr_inv = np.array([[1 / s2, 0, cr2], [0, 1 / s2, cc2], [0, 0, 1.0]])
    P = Tr_inv @ M @ Ts
    return P / P[2, 2]


def ransac(cps: np.ndarray, words: np.ndarray, model: int, threshold: float, n_refine: int,
           Hs: int, Ws: int, Hr: int, Wr: int, prior=None):
    """Returns (cps with updated flags, result dict): counts per hypothesis,
    the best index, the final inlier mask over candidates, the model in
    normalised and in pixel coordinates, and the candidate indices."""
    k = SAMPLE[model]
    words = np.asarray(words, dtype=np.uint32).reshape(-1, k)
    nh = len(words)
    cps = cps.copy()
    idx, src_px, dst_px = candidates(cps, prior)
    n = len(idx)
    src = normalise(src_px, Hs, Ws)
    dst = normalise(dst_px, Hr, Wr)
    s_ref = 0.5 * max(Hr, Wr)
    counts = np.full(nh, -1, np.int64)
    models = [None] * nh
    if n >= k:
        for h in range(nh):
            sel = sample_indices(words[h], n)
            if degenerate(src, dst, sel):
                continue
            M = fit(model, src[sel], dst[sel])
            if M is None:
                continue
            models[h] = M
            counts[h] = int(np.sum(residuals(M, src, dst, s_ref) <= threshold))
    res = dict(counts=counts, models=models, cand=idx, n_cand=n, best=-1, model=None, model_px=None,
               inliers=np.zeros(n, bool), residuals=None)
    elig = idx
    cps["flags"][elig] &= ~np.uint32(VALID | INCONSISTENT)
    if n < k or counts.max(initial=-1) < 0:
        cps["flags"][elig] |= INCONSISTENT
        return cps, res
    best = int(np.argmax(counts))          # first maximum: lowest index on ties
    M = models[best]
    inl = residuals(M, src, dst, s_ref) <= threshold
    for _ in range(n_refine):
        if inl.sum() < k:
            break
        M2 = fit(model, src[inl], dst[inl])
        if M2 is None:
            break
        M = M2
        inl = residuals(M, src, dst, s_ref) <= threshold
    r = residuals(M, src, dst, s_ref)
    inl = r <= threshold
    cps["flags"][elig[inl]] |= VALID
    cps["flags"][elig[~inl]] |= INCONSISTENT
    res.update(best=best, model=M, model_px=to_pixels(M, Hs, Ws, Hr, Wr), inliers=inl, residuals=r)
    return cps, res
