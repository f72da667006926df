"""Helpers shared by the GPU parity tests (comparison logic only)."""
import math

import numpy as np

from oracle import sfoc_oracle as O

# Tolerances (the figures the method is held to on the GPU).
NCC_TOL = 1e-4          # NCC scores: |gpu - oracle| <= 1e-4 (NCC lies in [-1, 1])
SUBPX_TOL = 0.05        # sub-pixel offsets, px
DESC_TOL = 1e-5         # float32 descriptors: |gpu - oracle| <= 1e-5 (values in [0, 1])
AMBIG_REL = 2e-4        # a second index within this fraction of the peak is a tie
CONSIST_BAND = 0.1      # |deviation - 1.5| below this may flip INCONSISTENT / VALID


def to_chw(F):
    return np.ascontiguousarray(np.asarray(F).transpose(2, 0, 1))


def compare_cps(g, o, surf_o, r, surf_g=None, check_consistency=True):
    """g: GPU records (structured), o: oracle records, surf_o: oracle surfaces.

    Integer CPs must agree exactly unless the oracle's surface holds the
    GPU's location within AMBIG_REL of its peak (several correct answers).
    Returns a dict of statistics."""
    V = 2 * r + 1
    n = len(o)
    stats = dict(n=n, ambiguous=0, max_score_err=0.0, max_sub_err=0.0, max_ncc_err=0.0, flips=0)
    base_mask = ~np.uint32(O.VALID | O.INCONSISTENT)
    for i in range(n):
        fo, fg = int(o["flags"][i]), int(g["flags"][i])
        assert (fo & int(base_mask)) == (fg & int(base_mask)), (i, fo, fg)
        if fo & (O.OOB | O.FLAT_T | O.FLAT_S | O.NONFINITE):
            assert g["dy"][i] == 0 and g["dx"][i] == 0 and g["score"][i] == 0
            continue
        if (g["dy"][i], g["dx"][i]) != (o["dy"][i], o["dx"][i]):
            ui, vi = o["dy"][i] + r, o["dx"][i] + r
            ug, vg = g["dy"][i] + r, g["dx"][i] + r
            pk = surf_o[i][ui, vi]
            assert abs(surf_o[i][ug, vg] - pk) <= AMBIG_REL * abs(pk) + NCC_TOL, (i, o[i], g[i])
            stats["ambiguous"] += 1
            continue
        stats["max_score_err"] = max(stats["max_score_err"], abs(float(g["score"][i]) - float(o["score"][i])))
        assert abs(float(g["score"][i]) - float(o["score"][i])) <= NCC_TOL * max(1.0, abs(float(o["score"][i])))
        e = max(abs(float(g["sub_dy"][i]) - o["sub_dy"][i]), abs(float(g["sub_dx"][i]) - o["sub_dx"][i]))
        stats["max_sub_err"] = max(stats["max_sub_err"], e)
        assert e <= SUBPX_TOL, (i, o[i], g[i])
        if check_consistency and (fo != fg):
            stats["flips"] += 1
    if surf_g is not None:
        stats["max_ncc_err"] = float(np.abs(np.asarray(surf_g, np.float64) - surf_o).max())
        assert stats["max_ncc_err"] <= NCC_TOL, stats
    return stats


def consistency_flip_allowed(o, priors=None):
    """Indices whose deviation from the oracle's median lies within
    CONSIST_BAND of the 1.5 px threshold."""
    bad = O.OOB | O.FLAT_T | O.FLAT_S | O.EDGE_PEAK | O.NONFINITE
    elig = (o["flags"] & bad) == 0
    if not elig.any():
        return set()
    py = np.zeros(len(o)) if priors is None else priors[:, 0]
    px = np.zeros(len(o)) if priors is None else priors[:, 1]
    ty = py + o["dy"] + o["sub_dy"]
    tx = px + o["dx"] + o["sub_dx"]
    dev = np.hypot(ty - np.median(ty[elig]), tx - np.median(tx[elig]))
    return set(np.nonzero(elig & (np.abs(dev - O.CONSISTENCY_PX) < CONSIST_BAND))[0].tolist())


def bf16_ulp(x):
    a = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(a, 1e-30)))
    return np.where(a > 0, 2.0 ** (e - 7), 2.0 ** -133)


def f16_ulp(x):
    a = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
    return 2.0 ** (e - 10)


def desc_condition(img, op):
    """Per-pixel, per-channel amplification of float32 rounding in the
    descriptor.  The absolute error of the smoothed map D is set by the scale
    of smooth(|F|) (F the signed steered response); normalisation divides it
    by the pixel's order norm sqrt(sum D^2 + eps).  Returns
    max(1, max(median, local) ||smooth(|F|)|| / sqrt(||D||^2 + eps)), which is
    about 1 for |.| rectification on textured images and large where signed
    responses cancel or a ReLU leaves an order block near zero."""
    import dataclasses
    img = np.asarray(img, np.float64)
    A, Q = O.sfoc_unnormalised(img, dataclasses.replace(op, rectify="signed"))
    H, W = img.shape
    N = op.n_orient
    if op.rectify == "abs":
        R = np.abs(A)
    elif op.rectify == "relu":
        R = np.maximum(A, 0.0)
    else:
        R = A
    sm = lambda X, c: O.dilated_smooth(X, Q, H, W, op.sd1 if c < N else op.sd2, op.K, op.dil)
    D = np.stack([sm(R[c], c) for c in range(A.shape[0])])
    Da = np.stack([sm(np.abs(A[c]), c) for c in range(A.shape[0])])
    kap = np.empty_like(D)
    for lo in range(0, D.shape[0], N):
        mag = np.sqrt((Da[lo:lo + N] ** 2).sum(axis=0))
        den = np.sqrt((D[lo:lo + N] ** 2).sum(axis=0) + op.eps)
        kap[lo:lo + N] = np.maximum(1.0, np.maximum(np.median(mag), mag) / den)
    return kap
