"""Descriptor storage in BF16 / FP16 (FFT in FP32, integral images and the
variance subtraction in FP64) against the oracle on the same rounded
descriptors (O64q): element by element on small pairs; on the 10000 x 10000
precision workload every one of the 5000 CPs against the oracle's stored
decisions (tests/golden/make_oracle_cps.py large), and sampled CPs with
their whole surfaces against the oracle recomputed live.  Per-CP NCC and
displacement errors against the unrounded oracle (O64) are reported and
written to gpurun_out/precision_large_errors.json."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import sfoc_oracle as O
from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth
from tests.gpu_util import (SUBPX_TOL, compare_cps, compare_to_golden, consistency_flip_allowed, golden_records,
                            load_golden)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DT = {"bf16": S.DTYPE_BF16, "f16": S.DTYPE_F16}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_small_pairs_rounded_storage(kind, seed):
    say("precision small", kind, seed)
    pr, ips, m, r = synth.workload(synth.SMALL, seed)
    p = S.preset("baseline", dtype=DT[kind])
    cps, ncc = S.register_cps(dev(pr.ref), dev(pr.sen), dev(ips), m, r, p, want_ncc=True)
    torch.cuda.synchronize()
    g = S.cps_to_numpy(cps)
    oq, sq = O.register_cps(pr.ref, pr.sen, ips, m, r, O.Params(), quantise=kind, want_surfaces=True)
    st = compare_cps(g, oq, sq, r, ncc.cpu().numpy())
    flips = {i for i in range(len(oq)) if oq["flags"][i] != g["flags"][i]}
    assert flips <= consistency_flip_allowed(oq)
    o, so = O.register_cps(pr.ref, pr.sen, ips, m, r, O.Params(), want_surfaces=True)
    ok = (o["flags"] & (O.OOB | O.FLAT_T | O.FLAT_S | O.NONFINITE)) == 0
    say("  vs O64q", st, "| vs O64: max NCC err %.2e, integer CPs equal %d/%d" % (
        np.abs(ncc.cpu().numpy() - so).max(), int(np.sum((g["dy"] == o["dy"]) & (g["dx"] == o["dx"]) & ok)),
        int(ok.sum())))


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_direct_form_per_window_integrals(kind):
    """Small windows with 16-bit storage take the direct form (R_ST summed
    in space on the matrix cores) by default: the match call with the
    reference's integral images and with per-window ones (NULL) against the
    oracle on the rounded descriptors, prior included."""
    say("direct form, single pair", kind)
    pr, ips, m, r = synth.workload(synth.SMALL, 5)
    prior = np.random.default_rng(4).integers(-2, 3, ips.shape).astype(np.int32)
    p = S.preset("baseline", dtype=DT[kind])
    Fr, i1, i2 = S.describe(dev(pr.ref), p)
    Fs, _, _ = S.describe(dev(pr.sen), p, integrals=False)
    oq, sq = O.register_cps(pr.ref, pr.sen, ips, m, r, O.Params(), quantise=kind, prior=prior,
                            want_surfaces=True)
    for integ in ((i1, i2), (None, None)):
        cps, ncc = S.fastncc_match(Fs, Fr, integ[0], integ[1], dev(ips), m, r, prior=dev(prior), want_ncc=True)
        torch.cuda.synchronize()
        g = S.cps_to_numpy(cps)
        st = compare_cps(g, oq, sq, r, ncc.cpu().numpy())
        flips = {i for i in range(len(oq)) if oq["flags"][i] != g["flags"][i]}
        assert flips <= consistency_flip_allowed(oq, prior)
        say("  integral images", "reference" if integ[0] is not None else "per window", st)


@pytest.fixture(scope="module")
def large():
    say("generating the 10000 x 10000 pair")
    pr, ips, m, r = synth.workload(synth.LARGE, 0)
    out = {}
    ref, sen, dips = dev(pr.ref), dev(pr.sen), dev(ips)
    for kind in ("bf16", "f16"):
        say("  GPU", kind)
        p = S.preset("baseline", dtype=DT[kind])
        R = S.Registrar(10000, 10000, 10000, 10000, len(ips), m, r, p, want_ncc=True)
        cps = R(ref, sen, dips)
        torch.cuda.synchronize()
        out[kind] = (S.cps_to_numpy(cps).copy(), R.ncc.cpu().numpy())
        del R
        torch.cuda.empty_cache()
    return pr, ips, m, r, out


def test_large_properties(large):
    pr, ips, m, r, out = large
    assert len(ips) == 5000
    for kind, (g, s) in out.items():
        assert np.all(np.abs(s) <= 1 + 1e-4)
        valid = (g["flags"] & O.VALID) != 0
        err = np.hypot(g["dy"] + g["sub_dy"] - pr.shift[0], g["dx"] + g["sub_dx"] - pr.shift[1])
        say(kind, "valid", int(valid.sum()), "correct@1.5px among valid", int((err[valid] <= 1.5).sum()))
        assert (err[valid] <= 1.5).mean() > 0.9
    a, b = out["bf16"][0], out["f16"][0]
    say("bf16 vs f16 integer CPs equal:", int(np.sum((a["dy"] == b["dy"]) & (a["dx"] == b["dx"]))), "of", len(a))


def test_large_all_cps_match_stored_oracle(large):
    """All 5000 CPs of both storages against the oracle on the same rounded
    descriptors: integer CPs equal (or another index of the oracle's tie set
    with the same refined displacement), scores within 1e-4, sub-pixel within
    0.05 px, flags equal.  Errors against the unrounded oracle are reported."""
    pr, ips, m, r, out = large
    gold = load_golden("large")
    from tests.golden.make_oracle_cps import input_digest
    assert str(gold["digest"]) == input_digest(pr.ref, pr.sen, ips), "regenerated inputs differ from the stored ones"
    o64, _ = golden_records(gold, "o64")
    report = {"workload": "10000x10000 pair, 5000 IPs, m 64, r 48, baseline SFOC", "kinds": {}}
    for kind, (g, s) in out.items():
        oq, ties = golden_records(gold, kind)
        gk = g.copy()
        gk["flags"] &= ~np.uint32(O.VALID | O.INCONSISTENT)
        st, score_err, off_err = compare_to_golden(gk, oq, ties, r, ref=o64)
        same64 = np.isfinite(score_err)
        summ = dict(st, vs_o64={
            "integer_equal": int(same64.sum()),
            "max_score_err": float(np.nanmax(score_err)), "median_score_err": float(np.nanmedian(score_err)),
            "max_offset_err_px": float(np.nanmax(off_err)), "median_offset_err_px": float(np.nanmedian(off_err)),
            "offset_err_gt_0p05": int(np.sum(off_err > SUBPX_TOL))})
        say(kind, summ)
        report["kinds"][kind] = dict(summ, score_err_vs_o64=[None if not np.isfinite(x) else float(x) for x in score_err],
                                     offset_err_vs_o64=[None if not np.isfinite(x) else float(x) for x in off_err])
        assert st["compared"] == st["equal"] + st["ambiguous_taken"]
    od = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    os.makedirs(od, exist_ok=True)
    with open(os.path.join(od, "precision_large_errors.json"), "w") as f:
        json.dump(report, f)


@pytest.mark.parametrize("k", [0, 2500, 4999])
def test_large_sampled_cps_live_oracle(large, k):
    """Whole surfaces of sampled CPs against the oracle computed live; the
    stored decisions are this oracle's."""
    pr, ips, m, r, out = large
    gold = load_golden("large")
    res = O.match_one_region_variants(pr.ref, pr.sen, ips[k], m, r, O.Params(), quantise=(None, "bf16", "f16"))
    for j, kind in enumerate(("o64", "bf16", "f16")):
        go, _ = golden_records(gold, kind)
        rec = res[j][0]
        assert (go["dy"][k], go["dx"][k], go["flags"][k]) == (rec[0], rec[1], rec[5])
        assert abs(go["score"][k] - rec[4]) <= 1e-12
    for j, kind in ((1, "bf16"), (2, "f16")):
        g, s = out[kind]
        rec, sq = res[j]
        oq = np.zeros(1, dtype=O.CP_DTYPE)
        oq["dy"], oq["dx"], oq["sub_dy"], oq["sub_dx"], oq["score"], oq["flags"] = rec
        gk = g[k:k + 1].copy()
        gk["flags"] &= ~np.uint32(O.VALID | O.INCONSISTENT)
        st = compare_cps(gk, oq, sq[None], r, s[k:k + 1], check_consistency=False)
        say(kind, k, "vs O64q", st, "| vs O64: NCC err %.2e" % np.abs(s[k] - res[0][1]).max())
