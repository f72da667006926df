"""Block-based FAST on the GPU (through the C ABI) against the FAST oracle:
bit-exact interest points, strengths and per-block counts on structured
random images of ragged sizes, on a 2048 x 2048 synthetic sensed image and
on sampled blocks of the 10000 x 10000 throughput configuration, the empty
cases, and registration from the detected points."""
import sys

import numpy as np
import pytest
from scipy import ndimage

from oracle import fast_oracle as F
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


def structured(seed, H, W):
    rng = np.random.default_rng(seed)
    a = ndimage.gaussian_filter(rng.uniform(0, 1, (H, W)), 1.5)
    for _ in range(max(4, H * W // 2000)):
        y0, x0 = rng.integers(0, H), rng.integers(0, W)
        a[y0:y0 + rng.integers(4, 30), x0:x0 + rng.integers(4, 30)] += rng.uniform(-0.4, 0.4)
    return a.astype(np.float32)


def run(img, thr, margin, nby, nbx, per, pad=0):
    H, W = img.shape
    buf = np.zeros((H, W + pad), np.float32)
    buf[:, :W] = img
    d = torch.from_numpy(buf).cuda()[:, :W]
    D = S.Detector(H, W, nby, nbx, per, thr, margin)
    ips, sc, cnt, n = D(d)
    k = int(n.item())
    return ips[:k].cpu().numpy(), sc[:k].cpu().numpy(), cnt.cpu().numpy()


@pytest.mark.parametrize("H,W,thr,margin,nby,nbx,per,pad", [
    (64, 64, 0.02, 0, 1, 1, 1, 0),
    (97, 131, 0.01, 5, 3, 4, 3, 7),
    (200, 170, 0.005, 20, 5, 5, 8, 0),
    (333, 257, 0.0, 12, 7, 3, 17, 3),
    (150, 300, 0.01, 40, 2, 6, 32, 0),
    (40, 1030, 0.003, 3, 1, 9, 5, 1),
    (211, 173, 0.004, 9, 13, 11, 1, 2),       # one per block
    (90, 90, 0.002, 3, 70, 9, 1, 0),          # more blocks than region rows
])
def test_parity(H, W, thr, margin, nby, nbx, per, pad):
    img = structured(H * 7 + W, H, W)
    gi, gs, gc = run(img, thr, margin, nby, nbx, per, pad)
    oi, osc, oc = F.detect(img, thr, margin, nby, nbx, per)
    say(f"fast {H}x{W} thr={thr} margin={margin} blocks={nby}x{nbx} per={per}: {len(oi)} IPs")
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gs, osc)


def test_empty_cases():
    img = structured(1, 50, 60)
    gi, gs, gc = run(img, 0.01, 30, 2, 2, 4)            # region empty (2 * 30 > 50)
    assert len(gi) == 0 and (gc == 0).all()
    gi, gs, gc = run(np.full((40, 40), 0.5, np.float32), 0.0, 3, 2, 2, 4)   # uniform: V = 0, not > 0
    assert len(gi) == 0
    gi, gs, gc = run(img, 10.0, 3, 3, 3, 2)             # threshold above every strength
    assert len(gi) == 0
    gi, gs, gc = run(img, 0.001, 3, 40, 50, 1)          # more blocks than region rows / columns
    oi, osc, oc = F.detect(img, 0.001, 3, 40, 50, 1)
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gi, oi)


def test_large_sampled_blocks():
    """The benchmark's throughput configuration (10000 x 10000 smoothed
    noise, 71 x 71 blocks, one point each, margin 80): the four corner blocks
    and eight random ones against the oracle run on a crop that holds the
    block, its suppression ring and the circle's reach (4 pixels), with the
    strengths outside the detection region removed as in the full image."""
    side, nb, thr, margin = 10000, 71, 0.002, 80
    gen = torch.Generator(device="cuda").manual_seed(0)
    big = torch.rand((1, 1, side, side), dtype=torch.float32, device="cuda", generator=gen)
    box = torch.full((1, 1, 5, 5), 1.0 / 25.0, dtype=torch.float32, device="cuda")
    conv = torch.nn.functional.conv2d
    big = conv(conv(big, box, padding=2), box, padding=2)[0, 0].contiguous()
    D = S.Detector(side, side, nb, nb, 1, thr, margin)
    ips, sc, cnt, n = D(big)
    torch.cuda.synchronize()
    k = int(n.item())
    ips, sc, cnt = ips[:k].cpu().numpy(), sc[:k].cpu().numpy(), cnt.cpu().numpy()
    img = big.cpu().numpy()
    b = max(3, margin)
    ys = F.block_bounds(b, side - 2 * b, nb)
    xs = F.block_bounds(b, side - 2 * b, nb)
    start = np.concatenate([[0], np.cumsum(cnt)])
    rng = np.random.default_rng(0)
    picks = [(0, 0), (0, nb - 1), (nb - 1, 0), (nb - 1, nb - 1)] + \
            [tuple(int(v) for v in rng.integers(0, nb, 2)) for _ in range(8)]
    h = 4
    for i, j in picks:
        y0, y1, x0, x1 = ys[i], ys[i + 1], xs[j], xs[j + 1]
        crop = img[y0 - h:y1 + h, x0 - h:x1 + h]
        V = F.strength(crop, 3)
        gy = np.arange(crop.shape[0])[:, None] + (y0 - h)
        gx = np.arange(crop.shape[1])[None, :] + (x0 - h)
        V[(gy < b) | (gy >= side - b) | (gx < b) | (gx >= side - b)] = -np.inf
        keep = F.suppress(V, thr)[h:h + y1 - y0, h:h + x1 - x0]
        vb = V[h:h + y1 - y0, h:h + x1 - x0]
        blk = i * nb + j
        cand = np.argwhere(keep)
        say(f"block ({i},{j}): {len(cand)} kept corners")
        if len(cand) == 0:
            assert cnt[blk] == 0
            continue
        vals = vb[cand[:, 0], cand[:, 1]]
        order = np.lexsort((cand[:, 0] * side + cand[:, 1], -vals.astype(np.float64)))
        best = cand[order[0]]
        assert cnt[blk] == 1
        assert tuple(ips[start[blk]]) == (y0 + best[0], x0 + best[1])
        assert sc[start[blk]] == vb[best[0], best[1]]


def test_scene_sensed_image():
    """The 2048 x 2048 sensed image of the benchmark pair: 20 x 20 blocks,
    one interest point each, inside the matching margin."""
    pr, _, m, r = synth.workload(synth.SCENE, 0)
    margin = (m + 1) // 2 + r
    gi, gs, gc = run(pr.sen, 0.05, margin, 20, 20, 1)
    oi, osc, oc = F.detect(pr.sen, 0.05, margin, 20, 20, 1)
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gi, oi)
    np.testing.assert_array_equal(gs, osc)
    say(f"scene: {len(gi)} IPs from 400 blocks")
    assert len(gi) >= 390


def test_registration_from_detected_points():
    pr, _, m, r = synth.workload(synth.SCENE, 0)
    margin = (m + 1) // 2 + r
    sen = torch.from_numpy(pr.sen).cuda()
    ips, _, _ = S.detect_ips(sen, 0.05, margin, 20, 20, 1)
    cps = S.cps_to_numpy(S.register_cps(torch.from_numpy(pr.ref).cuda(), sen, ips, m, r, S.preset("baseline")))
    v = (cps["flags"] & S.VALID) != 0
    err = np.hypot(cps["dy"] + cps["sub_dy"] - pr.shift[0], cps["dx"] + cps["sub_dx"] - pr.shift[1])
    say(f"detected IPs: {len(cps)}, VALID {int(v.sum())}, correct {int((err[v] <= 1.5).sum())}")
    assert v.sum() >= 0.6 * len(cps) and (err[v] <= 1.5).mean() >= 0.98
