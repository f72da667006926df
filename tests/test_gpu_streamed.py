"""The pair call streamed over bands of rows (sfoc_register_cps_streamed)
against the pair call on the whole images: the same integer CPs, flags and
records, surfaces within float64 box-sum rounding, for band heights from one
row to more than the image, priors, out-of-bounds IPs, float32 and bfloat16
storage (the latter on a window small enough for the direct form)."""
import sys

import numpy as np
import pytest

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth
from tests.gpu_util import AMBIG_REL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def case(seed, m, r, n=150):
    pr = synth.make_pair(seed, (700, 520), 5.0)
    ref = pr.ref
    sen = np.ascontiguousarray(pr.sen[:680, :500])
    ips = synth.random_ips(seed, 680, 500, n, 0)
    ips = np.concatenate([ips, np.array([[0, 0], [679, 250], [-40, 10], [900, 100]], np.int32)])
    ips = ips[np.argsort(ips[:, 0], kind="stable")]
    prior = np.random.default_rng(seed).integers(-6, 7, size=ips.shape).astype(np.int32)
    return ref, sen, ips, prior


def check_same(cw, nw, cs, ns, r):
    gw, gs = S.cps_to_numpy(cw), S.cps_to_numpy(cs)
    np.testing.assert_array_equal(gw["sen_row"], gs["sen_row"])
    np.testing.assert_array_equal(gw["sen_col"], gs["sen_col"])
    np.testing.assert_array_equal(gw["flags"], gs["flags"])
    V = 2 * r + 1
    nw, ns = nw.cpu().numpy(), ns.cpu().numpy()
    assert np.abs(nw - ns).max() <= 1e-5
    for i in np.nonzero((gw["dy"] != gs["dy"]) | (gw["dx"] != gs["dx"]))[0]:
        # only a tie of the whole-image surface may resolve the other way
        s = nw[i].ravel()
        a = (gw["dy"][i] + r) * V + gw["dx"][i] + r
        b = (gs["dy"][i] + r) * V + gs["dx"][i] + r
        assert s[b] >= s[a] - AMBIG_REL * abs(s[a]), i
    same = (gw["dy"] == gs["dy"]) & (gw["dx"] == gs["dx"])
    assert np.abs(gw["score"][same] - gs["score"][same]).max(initial=0.0) <= 1e-5
    assert np.abs(gw["sub_dy"][same] - gs["sub_dy"][same]).max(initial=0.0) <= 1e-3
    return int(same.sum())


@pytest.mark.parametrize("dtype,m,r", [(S.DTYPE_F32, 40, 12), (S.DTYPE_BF16, 24, 6)])
def test_streamed_equals_whole(dtype, m, r):
    ref, sen, ips, prior = case(11, m, r)
    p = S.preset("baseline", dtype=dtype)
    dr, ds, dips, dprior = dev(ref), dev(sen), dev(ips), dev(prior)
    cw, nw = S.register_cps(dr, ds, dips, m, r, p, prior=dprior, want_ncc=True)
    torch.cuda.synchronize()
    whole = S.register_workspace(700, 520, 680, 500, len(ips), m, r, p)
    for band in (1, 37, 128, 5000):
        say("streamed", dtype, m, r, "band rows", band)
        R = S.StreamedRegistrar(700, 520, 680, 500, len(ips), m, r, p, band_rows=band, max_prior=6,
                                want_ncc=True)
        cs = R(dr, ds, dips, dprior)
        torch.cuda.synchronize()
        same = check_same(cw, nw, cs, R.ncc, r)
        say("  integer CPs equal", same, "of", len(ips), "workspace", R.wsb, "vs whole", whole)
        if band < 200:
            assert R.wsb < whole
        # a second call on the same workspace gives the same records
        cs2 = R(dr, ds, dips, dprior).clone()
        torch.cuda.synchronize()
        assert torch.equal(cs2.cpu(), cs.cpu())


def test_streamed_without_prior_and_rejections():
    m, r = 32, 10
    ref, sen, ips, _ = case(12, m, r, n=60)
    p = S.preset("baseline")
    dr, ds, dips = dev(ref), dev(sen), dev(ips)
    cw, nw = S.register_cps(dr, ds, dips, m, r, p, want_ncc=True)
    R = S.StreamedRegistrar(700, 520, 680, 500, len(ips), m, r, p, band_rows=50, want_ncc=True)
    cs = R(dr, ds, dips)
    torch.cuda.synchronize()
    check_same(cw, nw, cs, R.ncc, r)
    # IPs out of row order, and a prior beyond max_prior, are refused before any launch
    rev = dev(np.ascontiguousarray(ips[::-1]))
    with pytest.raises(S.SfocError):
        R(dr, ds, rev)
    big = np.zeros_like(ips)
    big[3, 0] = 1
    with pytest.raises(S.SfocError):
        R(dr, ds, dips, dev(big))
