"""Descriptor storage in BF16 / FP16 (FFT in FP32, integral images and the
variance subtraction in FP64) against the oracle on the same rounded
descriptors (O64q), element by element on small pairs and on sampled CPs of
the 10000 x 10000 precision workload; errors against the unrounded oracle
(O64) are reported."""
import sys

import numpy as np
import pytest

from oracle import sfoc_oracle as O
from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth
from tests.gpu_util import compare_cps, consistency_flip_allowed

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


@pytest.mark.parametrize("k", [0, 70, 2500, 4999, 1234, 3777])
def test_large_sampled_cps(large, k):
    pr, ips, m, r, out = large
    for kind, (g, s) in out.items():
        rec, sq = O.match_one_region(pr.ref, pr.sen, ips[k], m, r, O.Params(), quantise=kind)
        oq = np.zeros(1, dtype=O.CP_DTYPE)
        oq["dy"], oq["dx"], oq["sub_dy"], oq["sub_dx"], oq["score"], oq["flags"] = rec
        gk = g[k:k + 1].copy()
        gk["flags"] &= ~np.uint32(O.VALID | O.INCONSISTENT)
        st = compare_cps(gk, oq, sq[None], r, s[k:k + 1], check_consistency=False)
        rec0, s0 = O.match_one_region(pr.ref, pr.sen, ips[k], m, r, O.Params())
        say(kind, k, "vs O64q", st, "| vs O64: NCC err %.2e, offset err %.3f px" % (
            np.abs(s[k] - s0).max(),
            np.hypot(gk["dy"][0] + gk["sub_dy"][0] - rec0[0] - rec0[2], gk["dx"][0] + gk["sub_dx"][0] - rec0[1] - rec0[3])))
