"""Noise sensitivity of the matching (Section 4.3) and the F-SFOC ablation
(Section 4.2: SFOC without its second-order channels).

Seeded pairs get Gaussian white noise or speckle on the sensed image at
the paper's levels; interest points come from block-based FAST on the noisy
sensed image, CPs from Fast-NCC with 80 x 80 templates, all in libsfoc's
kernels.  The score is the correct matching ratio CMR = NCM / total matches
(Section 4.1): total matches are the CPs with an interior peak (before any
outlier rejection), NCM those within 1.5 px of the known shift.

    python -m paper_2202_13347_amd.sweep --pairs 8 --out sweep.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth

CORRECT_PX = 1.5


def cmr(cps: np.ndarray, shift, prior=None) -> tuple[int, int]:
    """(NCM, total matches) of CP records against a known shift (dy, dx)."""
    peak = (cps["flags"] & (S.VALID | S.INCONSISTENT)) != 0
    py = 0 if prior is None else prior[:, 0]
    px = 0 if prior is None else prior[:, 1]
    dy = py + cps["dy"] + cps["sub_dy"].astype(np.float64)
    dx = px + cps["dx"] + cps["sub_dx"].astype(np.float64)
    ok = np.hypot(dy - shift[0], dx - shift[1]) <= CORRECT_PX
    return int((ok & peak).sum()), int(peak.sum())


NOISE = {"gaussian": synth.gaussian_noise, "speckle": synth.speckle_noise}


def noisy_sensed(sen: np.ndarray, kind: str, v: float, pair_index: int) -> np.ndarray:
    """The sensed image of pair `pair_index` with noise of type `kind` and
    variance v, seeded per pair and level (v = 0: unchanged)."""
    return NOISE[kind](sen, v, 1000 * pair_index + int(round(v * 1e4))) if v > 0 else sen


def run(n_pairs: int | None = None, recipe: dict = synth.SWEEP, preset: str = "paper", device="cuda", log=None):
    """CMR (averaged over pairs, and pooled) per noise type and level, for
    SFOC and F-SFOC.  Returns a dict of tables and the GPU time spent."""
    import torch
    n_pairs = n_pairs or recipe["n_pairs"]
    m, r = recipe["m"], recipe["r"]
    margin = (m + 1) // 2 + r
    nby, nbx = recipe["blocks"]
    size = recipe["size"]
    pairs = [synth.sweep_pair(s, recipe) for s in range(n_pairs)]
    descs = {"SFOC": S.preset(preset)}
    f = S.preset(preset)
    f.second_order = 0
    descs["F-SFOC"] = f
    det = S.Detector(size, size, nby, nbx, 1, recipe["fast_threshold"], margin, device=device)
    regs = {k: S.Registrar(size, size, size, size, nby * nbx, m, r, p, device=device) for k, p in descs.items()}
    out = {"levels": {"gaussian": recipe["gaussian"], "speckle": recipe["speckle"]}, "pairs": n_pairs,
           "template": m, "radius": r, "size": size, "ips_per_pair": nby * nbx, "preset": preset}
    gpu_s = 0.0
    for kind, levels in (("gaussian", recipe["gaussian"]), ("speckle", recipe["speckle"])):
        tab = {k: [] for k in descs}
        pooled = {k: [] for k in descs}
        for v in levels:
            per = {k: [] for k in descs}
            tot = {k: [0, 0] for k in descs}
            for i, pr in enumerate(pairs):
                sen_np = noisy_sensed(pr.sen, kind, v, i)
                sen = torch.from_numpy(sen_np).to(device)
                ref = torch.from_numpy(pr.ref).to(device)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ips, _, _, n = det(sen)
                k_ips = int(n.item())
                ips[k_ips:] = -(1 << 20)    # unused capacity: out of the image, so OOB records
                res = {}
                for k, R in regs.items():
                    res[k] = R(ref, sen, ips)
                torch.cuda.synchronize()
                gpu_s += time.perf_counter() - t0
                for k in descs:
                    c = S.cps_to_numpy(res[k])[:k_ips]
                    ncm, total = cmr(c, pr.shift)
                    per[k].append(ncm / max(1, total))
                    tot[k][0] += ncm
                    tot[k][1] += total
            for k in descs:
                tab[k].append(float(np.mean(per[k])))
                pooled[k].append(tot[k][0] / max(1, tot[k][1]))
            if log:
                log(f"{kind} v={v}: " + ", ".join(f"{k} CMR {tab[k][-1]:.3f}" for k in descs))
        out[kind] = {"mean_cmr": tab, "pooled_cmr": pooled}
    out["gpu_s"] = gpu_s
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=synth.SWEEP["n_pairs"])
    ap.add_argument("--preset", default="paper")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.init()    # the GPU runtime is brought up by torch before the library's first call
    S.lib()
    res = run(args.pairs, preset=args.preset, log=lambda s: print(s, flush=True))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
