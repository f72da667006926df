"""Learned head on the GPU (through the C ABI) against the FP64 head oracle:
features, forward, gradients, Adam and the inference decision; determinism,
overfitting one batch, and the gain over the plain peak fit on held-out
seeds."""
import sys

import numpy as np
import pytest

from oracle import head_oracle as H
from oracle import sfoc_oracle as O
from paper_2202_13347_amd import head as HD
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_hwc(d):
    return d.float().permute(1, 2, 0).double().cpu().numpy()


@pytest.mark.parametrize("m,r,dtype,use_prior", [(32, 10, S.DTYPE_F32, False), (24, 20, S.DTYPE_F32, True),
                                                 (32, 18, S.DTYPE_BF16, False)])
def test_features_match_oracle(m, r, dtype, use_prior):
    say(f"features m={m} r={r} dtype={dtype}")
    pr = synth.make_pair(5, 256, max_shift=6.0)
    b = (m + 1) // 2 + r + 3
    ips = np.concatenate([synth.random_ips(5, 256, 256, 24, b), np.array([[3, 3]], np.int32)])
    prior = np.random.default_rng(5).integers(-3, 4, (len(ips), 2)).astype(np.int32) if use_prior else None
    p = S.preset("baseline", dtype=dtype)
    dref, i1, i2 = S.describe(dev(pr.ref), p)
    dsen, _, _ = S.describe(dev(pr.sen), p, integrals=False)
    dips = dev(ips)
    dprior = None if prior is None else dev(prior)
    cps, ncc = S.fastncc_match(dsen, dref, i1, i2, dips, m, r, prior=dprior, want_ncc=True)
    crops, stats = S.head_features(dsen, dref, i1, i2, dips, m, r, ncc, cps, prior=dprior)
    g = S.cps_to_numpy(cps)
    elig = H.eligible(g["flags"])
    assert elig.sum() >= 10 and not elig[-1]
    oc, ost = H.features(to_hwc(dsen), to_hwc(dref), ips, prior, m, r, g, ncc.cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(crops.cpu().numpy(), oc.astype(np.float32))
    np.testing.assert_allclose(stats.cpu().numpy(), ost, rtol=2e-6, atol=2e-7)


def _params(seed):
    th = synth.head_init_params(seed)
    th = th + np.random.default_rng(seed).normal(0, 0.02, th.shape).astype(np.float32)
    return th


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    crops = rng.uniform(-1, 1, (B, 33, 33)).astype(np.float32)
    crops[:, :, :4] = -1.0                              # padded border, as for small surfaces
    stats = rng.uniform(-1, 1, (B, 8)).astype(np.float32)
    label = (rng.random(B) < 0.6).astype(np.float32)
    target = rng.uniform(-0.6, 0.6, (B, 2)).astype(np.float32)
    return crops, stats, label, target


def test_forward_matches_oracle():
    th = _params(1)
    crops, stats, _, _ = _batch(2, 37)
    head = S.Head(th)
    out = head.forward(dev(crops), dev(stats)).cpu().numpy()
    want, _ = H.forward(th.astype(np.float64), crops, stats, quantise=True)
    np.testing.assert_allclose(out, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())


def _block_errors(g, want):
    errs = {}
    o = 0
    for name, shape in H.layout():
        n = int(np.prod(shape))
        a, b = g[o:o + n], want[o:o + n]
        errs[name] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12))
        o += n
    return errs


def test_gradients_match_oracle():
    th = _params(3)
    crops, stats, label, target = _batch(4, 45)
    head = S.Head(th)
    loss, grad = head.train_step(dev(crops), dev(stats), dev(label), dev(target), lr=0.0, want_grad=True)
    L, want = H.backward(th.astype(np.float64), crops, stats, label, target[:, 0], target[:, 1], quantise=True)
    assert float(loss) == pytest.approx(L, rel=1e-5)
    g = grad.cpu().numpy()
    errs = _block_errors(g, want)
    say("gradient relative errors", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-4, errs
    # lr = 0: parameters unchanged, moments = (0.1 g, 0.001 g^2)
    np.testing.assert_array_equal(head.params.cpu().numpy(), th)
    np.testing.assert_allclose(head.m.cpu().numpy(), 0.1 * g, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(head.v.cpu().numpy(), 0.001 * g * g, rtol=1e-5, atol=1e-15)


def test_adam_matches_oracle():
    th = _params(5)
    crops, stats, label, target = _batch(6, 32)
    head = S.Head(th)
    x = th.astype(np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    for t in range(1, 4):
        before = head.params.cpu().numpy().astype(np.float64)
        _, grad = head.train_step(dev(crops), dev(stats), dev(label), dev(target), lr=1e-3, want_grad=True)
        g = grad.cpu().numpy().astype(np.float64)
        x, m, v = H.adam_step(before, g, m, v, t, 1e-3)
        np.testing.assert_allclose(head.params.cpu().numpy(), x, rtol=0, atol=2e-6)


def test_training_is_deterministic():
    crops, stats, label, target = [dev(a) for a in _batch(7, 64)]
    res = []
    for _ in range(2):
        head = S.Head(_params(8))
        for _ in range(3):
            head.train_step(crops, stats, label, target, lr=1e-3)
        res.append(head.params.cpu().numpy())
    np.testing.assert_array_equal(res[0], res[1])


def test_overfits_one_batch():
    crops, stats, label, target = [dev(a) for a in _batch(9, 64)]
    head = S.Head(synth.head_init_params(10))
    first = None
    for k in range(300):
        loss, _ = head.train_step(crops, stats, label, target, lr=3e-3)
        if k == 0:
            first = float(loss)
    last = float(loss)
    say(f"overfit: loss {first:.4f} -> {last:.4f}")
    assert last < 0.1 * first


def test_infer_decision_matches_oracle():
    th = _params(11)
    crops, stats, _, _ = _batch(12, 40)
    c = np.zeros(40, dtype=S.CP_DTYPE)
    c["flags"] = np.array([S.VALID, S.INCONSISTENT, S.OOB, S.EDGE_PEAK, S.FLAT_S] * 8, np.uint32)
    c["dy"] = 1
    c["sub_dy"] = 0.25
    cps = dev(c.view(np.int32).reshape(40, 8))
    head = S.Head(th)
    out = head.infer(dev(crops), dev(stats), cps, threshold=0.5, want_out=True)
    g = S.cps_to_numpy(cps)
    oc = np.zeros(40, dtype=O.CP_DTYPE)
    for f in ("flags", "dy", "sub_dy"):
        oc[f] = c[f]
    want = H.apply(oc, out.cpu().numpy().astype(np.float64), 0.5)
    near = np.abs(out.cpu().numpy()[:, 0]) < 1e-6    # sigmoid at the threshold: either answer
    np.testing.assert_array_equal(g["flags"][~near], want["flags"][~near])
    np.testing.assert_array_equal(g["sub_dy"], want["sub_dy"].astype(np.float32))
    np.testing.assert_array_equal(g["sub_dx"], want["sub_dx"].astype(np.float32))
    assert (g["flags"][2::5] == S.OOB).all() and (g["sub_dy"][2::5] == 0.25).all()


def test_learned_head_gain():
    """Training run on seeded pairs with known shifts (about 60k samples),
    evaluated on held-out seeds.  Target: learned sub-pixel offsets within
    0.1 px (RMSE over correct CPs) of the parabola fit or better.  The
    learned validity is local to each CP while the consistency check uses
    the pair's median displacement; it must stay within 0.1 of the check's
    F1.  The figures are printed."""
    say("head gain: building samples")
    data = HD.build(range(HD.TRAIN_SEED0, HD.TRAIN_SEED0 + 600), workers=8)
    say(f"head gain: {int(data['label'].shape[0])} samples")
    head = S.Head(synth.head_init_params(0))
    hist = HD.train(head, data, epochs=6, batch=256, lr=2e-3, log=say)
    assert hist[-1] < hist[0]
    res = HD.evaluate(head, range(HD.TEST_SEED0, HD.TEST_SEED0 + 100), workers=8)
    say("head gain:", res)

    def f1(p, r):
        return 2 * p * r / max(p + r, 1e-12)

    assert res["rmse_learned"] <= res["rmse_plain"] + 0.1
    assert f1(res["precision_learned"], res["recall_learned"]) >= f1(res["precision_plain"], res["recall_plain"]) - 0.1


def test_shipped_parameters_gain():
    """The parameters shipped with the package (trained by
    `python -m paper_2202_13347_amd.head train`, 2000 pairs, 10 epochs) on
    held-out seeds: lower sub-pixel RMSE than the parabola fit."""
    head = S.Head(HD.load_params())
    res = HD.evaluate(head, range(HD.TEST_SEED0 + 500, HD.TEST_SEED0 + 580), workers=8)
    say("shipped head:", res)
    assert res["rmse_learned"] < res["rmse_plain"]
