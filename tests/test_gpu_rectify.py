"""Rectification on the GPU (through the C ABI) against the FP64 oracle:
element-wise on small and ragged images with padded pitches, sampled on a
large one, and the registration loop on warped pairs (RANSAC model ->
rectify -> matching again finds no displacement)."""
import sys

import numpy as np
import pytest

from oracle import rectify_oracle as X
from oracle import ransac_oracle as R
from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S.lib()
    yield
    torch.cuda.synchronize()


def models():
    return {
        "identity": np.eye(3),
        "translation": np.array([[1, 0, 3.25], [0, 1, -7.5], [0, 0, 1.0]]),
        "affine": np.array([[1.02, 0.03, -4.0], [-0.025, 0.97, 6.5], [0, 0, 1.0]]),
        "projective": np.array([[0.99, 0.01, 2.0], [0.02, 1.01, -3.0], [3e-4, -2e-4, 1.0]]),
        "horizon": np.array([[1, 0, 0], [0, 1, 0], [0, 0.02, 1.0]]),   # inverse w <= 0 from column 50
        "flip": np.array([[-1, 0, 60.0], [0, 1, 0], [0, 0, 1.0]]),     # negative determinant
    }


def near_boundary(M, Hs, Ws, Ho, Wo, tol=1e-6):
    py, px, ok = X.source_points(M, Ho, Wo)
    Minv = np.linalg.inv(M)
    r, c = np.meshgrid(np.arange(Ho, dtype=np.float64), np.arange(Wo, dtype=np.float64), indexing="ij")
    w = Minv[2, 0] * r + Minv[2, 1] * c + Minv[2, 2]
    edge = (np.abs(py) < tol) | (np.abs(py - (Hs - 1)) < tol) | (np.abs(px) < tol) | (np.abs(px - (Ws - 1)) < tol)
    return edge | (np.abs(w) < 1e-9)


@pytest.mark.parametrize("name", list(models()))
@pytest.mark.parametrize("Hs,Ws,Ho,Wo,pad_s,pad_o", [(64, 96, 70, 90, 0, 0), (57, 1031, 61, 1029, 5, 3),
                                                     (130, 2200, 120, 2100, 16, 0)])
def test_parity(name, Hs, Ws, Ho, Wo, pad_s, pad_o):
    M = models()[name]
    rng = np.random.default_rng(Hs + Wo)
    img = rng.uniform(-1, 1, (Hs, Ws + pad_s)).astype(np.float32)
    sen = torch.from_numpy(img).cuda()[:, :Ws]
    out = torch.full((Ho, Wo + pad_o), 123.0, dtype=torch.float32, device="cuda")[:, :Wo]
    S.rectify(sen, M, (Ho, Wo), fill=float("nan"), out=out)
    got = out.cpu().numpy()
    want = X.rectify(img[:, :Ws].astype(np.float64), M, Ho, Wo, fill=np.nan)
    skip = near_boundary(M, Hs, Ws, Ho, Wo)
    np.testing.assert_array_equal(np.isnan(got[~skip]), np.isnan(want[~skip]))
    fin = ~skip & ~np.isnan(want)
    assert fin.sum() > 0 or name == "horizon"
    np.testing.assert_allclose(got[fin], want[fin], rtol=0, atol=2e-6)
    say(f"rectify {name} {Hs}x{Ws}->{Ho}x{Wo}: {int(fin.sum())} compared, {int(skip.sum())} near the border")


def test_padding_untouched_and_fill_value():
    rng = np.random.default_rng(9)
    img = rng.uniform(0, 1, (40, 40)).astype(np.float32)
    buf = torch.full((30, 48), 5.0, dtype=torch.float32, device="cuda")
    M = np.array([[1, 0, 20.0], [0, 1, 0], [0, 0, 1.0]])   # output rows < 20 read sensed rows < 0: fill
    S.rectify(torch.from_numpy(img).cuda(), M, (30, 45), fill=-3.0, out=buf[:, :45])
    b = buf.cpu().numpy()
    assert (b[:, 45:] == 5.0).all()
    assert (b[:20, :40] == -3.0).all() and (b[:, 40:45] == -3.0).all()
    np.testing.assert_array_equal(b[20:30, :40], img[0:10, :40])


def test_large_sampled():
    """8192 x 6000 through a projective map; 20000 sampled output pixels
    against the oracle computed point by point."""
    H, W = 8192, 6000
    gen = torch.Generator(device="cuda").manual_seed(5)
    sen = torch.rand((H, W), dtype=torch.float32, device="cuda", generator=gen)
    M = np.array([[1.001, 0.004, -6.0], [-0.003, 0.999, 4.5], [2e-7, -1e-7, 1.0]])
    out = S.rectify(sen, M, (H, W), fill=0.0)
    rng = np.random.default_rng(6)
    rr = rng.integers(0, H, 20000)
    cc = rng.integers(0, W, 20000)
    Minv = np.linalg.inv(M)
    P = np.stack([rr, cc, np.ones_like(rr)], 1).astype(np.float64) @ Minv.T
    py, px = P[:, 0] / P[:, 2], P[:, 1] / P[:, 2]
    img = sen.cpu().numpy()
    want = X.bilinear(img, py, px, 0.0)
    got = out.cpu().numpy()[rr, cc]
    edge = (np.abs(py) < 1e-6) | (np.abs(py - (H - 1)) < 1e-6) | (np.abs(px) < 1e-6) | (np.abs(px - (W - 1)) < 1e-6)
    np.testing.assert_allclose(got[~edge], want[~edge], rtol=0, atol=2e-6)


@pytest.mark.parametrize("seed", [0])
def test_registration_loop(seed):
    """Warped pair: match, projective RANSAC, rectify the sensed image with
    the model; matching the rectified image against the reference again
    gives displacements within 1.5 px for the CPs RANSAC kept."""
    rec = synth.WARP
    w = synth.make_warp_pair(seed, rec)
    size, m, r = rec["size"], rec["m"], rec["r"]
    ips = synth.grid_ips(size, size, rec["n_side"], (m + 1) // 2 + r)
    p = S.preset("baseline")
    ref = torch.from_numpy(w.ref).cuda()
    dips = torch.from_numpy(ips).cuda()
    cps = S.register_cps(ref, torch.from_numpy(w.sen).cuda(), dips, m, r, p)
    RS = S.Ransac(len(ips), S.ransac_params(R.PROJECTIVE, 2048, (size, size, size, size), 1.5, 2))
    RS(cps, torch.from_numpy(synth.ransac_words(seed, 2048, 4).view(np.int32)).cuda())
    kept = (S.cps_to_numpy(cps)["flags"] & S.VALID) != 0
    rect = S.rectify(torch.from_numpy(w.sen).cuda(), RS.model, (size, size), fill=0.0)
    again = S.cps_to_numpy(S.register_cps(ref, rect, dips, m, r, p))
    d = np.hypot(again["dy"] + again["sub_dy"], again["dx"] + again["sub_dx"])
    ok = (again["flags"] & (S.VALID | S.INCONSISTENT)) != 0
    sel = kept & ok
    frac = float((d[sel] <= 1.5).mean())
    say(f"registration loop seed {seed}: {int(sel.sum())} CPs, {frac:.3f} within 1.5 px after rectification, "
        f"median |d| {float(np.median(d[sel])):.3f} px")
    assert sel.sum() > 200 and frac >= 0.95
