"""Helpers shared by the GPU parity tests (comparison logic only)."""
import math

import numpy as np

from oracle import sfoc_oracle as O

# Tolerances (the figures the method is held to on the GPU).
NCC_TOL = 1e-4          # NCC scores: |gpu - oracle| <= 1e-4 (NCC lies in [-1, 1])
SUBPX_TOL = 0.05        # sub-pixel offsets, px
DESC_TOL = 1e-5         # float32 descriptors: |gpu - oracle| <= 1e-5 (values in [0, 1])
AMBIG_REL = 2e-4        # a second index within this fraction of the peak is a tie
KAPPA_CAP_ABS = 32.0    # largest conditioning factor accepted under |.| rectification (measured <= 23.3)
CONSIST_BAND = 0.1      # |deviation - 1.5| below this may flip INCONSISTENT / VALID


def to_chw(F):
    return np.ascontiguousarray(np.asarray(F).transpose(2, 0, 1))


def near_peak(surf, idx):
    """Row-major indices of the surface whose value lies within AMBIG_REL *
    |peak| of the peak at `idx` (the tie set of the G13 reading; it always
    holds idx itself)."""
    s = np.asarray(surf, np.float64).ravel()
    pk = s[idx]
    return np.nonzero(s >= pk - AMBIG_REL * abs(pk))[0]


def total_offset_err(a, b):
    """Largest per-axis difference of the refined displacements dy + sub_dy,
    dx + sub_dx of two records."""
    return max(abs(float(a["dy"]) + float(a["sub_dy"]) - float(b["dy"]) - float(b["sub_dy"])),
               abs(float(a["dx"]) + float(a["sub_dx"]) - float(b["dx"]) - float(b["sub_dx"])))


def tie_on_border(a, b, r):
    """True when either of two tied records lies on the border of the
    (2r+1)^2 surface, where the peak gets no parabola refinement (its
    EDGE_PEAK flag is set), so their refined displacements need not agree."""
    return any(abs(int(x["dy"])) == r or abs(int(x["dx"])) == r for x in (a, b))


def load_golden(name):
    """Stored oracle CPs of a full-size workload (tests/golden/make_oracle_cps.py)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_cps_{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def golden_records(gold, kind):
    """(records, ties) of one storage kind of a golden file: records in the
    oracle's CP layout, ties a dict cp -> set of (dy, dx) also correct."""
    rec = gold[kind + "_rec"]
    o = np.zeros(len(rec), dtype=O.CP_DTYPE)
    o["dy"], o["dx"] = rec[:, 0].astype(np.int32), rec[:, 1].astype(np.int32)
    o["sub_dy"], o["sub_dx"], o["score"] = rec[:, 2], rec[:, 3], rec[:, 4]
    o["flags"] = gold[kind + "_flags"]
    ties = {}
    for i, dy, dx in gold[kind + "_ties"]:
        ties.setdefault(int(i), set()).add((int(dy), int(dx)))
    return o, ties


def compare_to_golden(g, o, ties, r, ref=None):
    """GPU records g against stored oracle records o (flags before the
    consistency check) with the same tie rule as compare_cps.  `ref`: the
    unrounded oracle's records, against which per-CP score and displacement
    errors are reported (not asserted).  Returns statistics and per-CP
    error arrays."""
    n = len(o)
    base_mask = int(~np.uint32(O.VALID | O.INCONSISTENT))
    st = dict(n=n, compared=0, equal=0, ambiguous=len(ties), ambiguous_taken=0, max_score_err=0.0,
              max_sub_err=0.0)
    score_err = np.full(n, np.nan)
    off_err = np.full(n, np.nan)
    for i in range(n):
        fo, fg = int(o["flags"][i]), int(g["flags"][i]) & base_mask
        if fo & (O.OOB | O.FLAT_T | O.FLAT_S | O.NONFINITE):
            assert fo == fg, (i, fo, fg)
            continue
        st["compared"] += 1
        same = (int(g["dy"][i]), int(g["dx"][i])) == (int(o["dy"][i]), int(o["dx"][i]))
        if not same:
            assert (int(g["dy"][i]), int(g["dx"][i])) in ties.get(i, ()), (i, o[i], g[i])
            if not tie_on_border(g[i], o[i], r):
                assert total_offset_err(g[i], o[i]) <= SUBPX_TOL, (i, o[i], g[i])
            st["ambiguous_taken"] += 1
        else:
            st["equal"] += 1
            assert fo == fg, (i, fo, fg)
            e = abs(float(g["score"][i]) - float(o["score"][i]))
            st["max_score_err"] = max(st["max_score_err"], e)
            assert e <= NCC_TOL, (i, o[i], g[i])
            e = max(abs(float(g["sub_dy"][i]) - o["sub_dy"][i]), abs(float(g["sub_dx"][i]) - o["sub_dx"][i]))
            st["max_sub_err"] = max(st["max_sub_err"], e)
            assert e <= SUBPX_TOL, (i, o[i], g[i])
        if ref is not None:
            if (int(g["dy"][i]), int(g["dx"][i])) == (int(ref["dy"][i]), int(ref["dx"][i])):
                score_err[i] = abs(float(g["score"][i]) - float(ref["score"][i]))
            off_err[i] = total_offset_err(g[i], ref[i])
    return st, score_err, off_err


def compare_cps(g, o, surf_o, r, surf_g=None, check_consistency=True):
    """g: GPU records (structured), o: oracle records, surf_o: oracle surfaces.

    A CP is ambiguous when the oracle surface holds a second index within
    AMBIG_REL * |peak| of its peak (the top-2 gap is below that); then any
    index of that tie set is a correct answer.  Every other CP must agree on
    the integer location exactly.  Returns statistics, among them
    `ambiguous` (oracle CPs with such a tie, whatever the GPU chose) and
    `ambiguous_taken` (those where the GPU took another index of the set)."""
    V = 2 * r + 1
    n = len(o)
    stats = dict(n=n, compared=0, ambiguous=0, ambiguous_taken=0, max_score_err=0.0, max_sub_err=0.0,
                 max_ncc_err=0.0, flips=0)
    base_mask = ~np.uint32(O.VALID | O.INCONSISTENT)
    for i in range(n):
        fo, fg = int(o["flags"][i]), int(g["flags"][i])
        if fo & (O.OOB | O.FLAT_T | O.FLAT_S | O.NONFINITE):
            assert (fo & int(base_mask)) == (fg & int(base_mask)), (i, fo, fg)
            assert g["dy"][i] == 0 and g["dx"][i] == 0 and g["score"][i] == 0
            continue
        stats["compared"] += 1
        io = (int(o["dy"][i]) + r) * V + int(o["dx"][i]) + r
        ig = (int(g["dy"][i]) + r) * V + int(g["dx"][i]) + r
        ties = near_peak(surf_o[i], io)
        if len(ties) > 1:
            stats["ambiguous"] += 1
            assert ig in ties, (i, o[i], g[i])
            if ig != io:
                # another correct integer answer: the refined displacement
                # must still agree, unless the other index lies on the
                # surface border (no refinement there, EDGE_PEAK instead)
                stats["ambiguous_taken"] += 1
                if not tie_on_border(g[i], o[i], r):
                    assert total_offset_err(g[i], o[i]) <= SUBPX_TOL, (i, o[i], g[i])
                continue
        assert ig == io, (i, o[i], g[i])
        assert (fo & int(base_mask)) == (fg & int(base_mask)), (i, fo, fg)
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
