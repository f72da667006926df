"""Pins of the head oracle against things other than itself: a library
correlation, finite differences, closed forms and brute force."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import head_oracle as H
from oracle import sfoc_oracle as O
from paper_2202_13347_amd import synth


def test_parameter_count():
    # conv1 32*9 + 32; conv2..4 3 * (32*32*9 + 32); fc1 32*(800 + 8) + 32; fc2 3*32 + 3
    assert H.N_PARAMS == 288 + 32 + 3 * (9216 + 32) + 32 * 808 + 32 + 96 + 3 == 54051
    th = synth.head_init_params(0)
    assert th.shape == (H.N_PARAMS,) and th.dtype == np.float32
    P = H.unpack(th)
    assert np.all(P["conv1.b"] == 0) and np.abs(P["conv2.w"]).max() <= np.sqrt(6 / 288)
    assert np.abs(P["fc1.w"]).max() <= np.sqrt(6 / 808) and np.abs(P["fc1.w"]).max() > 0.9 * np.sqrt(6 / 808)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_forward_is_a_correlation(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 7, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = H.conv_forward(x, w, b, stride)
    for n in range(2):
        for o in range(4):
            acc = np.full((7, 6), b[o])
            for c in range(3):
                acc = acc + correlate2d(np.pad(x[n, c], 1), w[o, c], mode="valid")
            np.testing.assert_allclose(got[n, o], acc[::stride, ::stride], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 2, 5, 5))
    w = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    R = rng.standard_normal(H.conv_forward(x, w, b, stride).shape)
    f = lambda x_, w_, b_: float((H.conv_forward(x_, w_, b_, stride) * R).sum())
    dx, dw, db = H.conv_backward(x, w, R, stride)
    h = 1e-6
    for arr, g in ((x, dx), (w, dw), (b, db)):
        for idx in list(np.ndindex(arr.shape))[::5]:
            e = np.zeros_like(arr)
            e[idx] = h
            args_p = [x, w, b]
            args_m = [x, w, b]
            k = [x is arr, w is arr, b is arr].index(True)
            args_p[k] = arr + e
            args_m[k] = arr - e
            fd = (f(*args_p) - f(*args_m)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def _batch(seed, B=3):
    rng = np.random.default_rng(seed)
    crops = rng.uniform(-1, 1, (B, 33, 33))
    stats = rng.uniform(-1, 1, (B, 8))
    y = np.array([1.0, 0.0, 1.0][:B])
    ty = rng.uniform(-0.5, 0.5, B)
    tx = rng.uniform(-0.5, 0.5, B)
    return crops, stats, y, ty, tx


def test_network_gradient_finite_differences():
    th = synth.head_init_params(3).astype(np.float64)
    th += np.random.default_rng(4).normal(0, 0.01, th.shape)   # non-zero biases
    crops, stats, y, ty, tx = _batch(5)
    L, g = H.backward(th, crops, stats, y, ty, tx, quantise=False)
    assert np.isfinite(L)
    rng = np.random.default_rng(6)
    offs, o = {}, 0
    for name, shape in H.layout():
        offs[name] = (o, int(np.prod(shape)))
        o += int(np.prod(shape))
    idx = []
    for name, (o, n) in offs.items():   # a few entries of every block
        idx += list(o + rng.choice(n, size=min(n, 6), replace=False))
    h = 1e-6
    worst = 0.0
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        lp = H.loss(H.forward(th + e, crops, stats, False)[0], y, ty, tx)
        lm = H.loss(H.forward(th - e, crops, stats, False)[0], y, ty, tx)
        fd = (lp - lm) / (2 * h)
        err = abs(fd - g[k]) / max(1e-3, abs(fd))
        worst = max(worst, err)
        assert err <= 1e-5, (k, fd, g[k])


def test_quantised_gradient_is_straight_through():
    th = synth.head_init_params(7).astype(np.float64)
    crops, stats, y, ty, tx = _batch(8)
    L1, g1 = H.backward(th, crops, stats, y, ty, tx, quantise=True)
    P = H.unpack(th.copy())
    q = {k: (O.round_to_bf16(v) if k.endswith(".w") else v) for k, v in P.items()}
    L2, g2 = H.backward(H.pack(q), crops, stats, y, ty, tx, quantise=False)
    assert L1 == pytest.approx(L2, rel=1e-14)
    np.testing.assert_allclose(g1, g2, rtol=1e-12, atol=1e-15)


def test_bce_and_smooth_l1_closed_forms():
    l = np.array([-3.0, -0.2, 0.0, 0.7, 4.0])
    for y in (0.0, 1.0):
        s = 1 / (1 + np.exp(-l))
        np.testing.assert_allclose(H.bce_with_logits(l, y), -(y * np.log(s) + (1 - y) * np.log(1 - s)), rtol=1e-12)
    assert np.isfinite(H.bce_with_logits(np.array([800.0, -800.0]), 1.0)).all()
    assert H.bce_with_logits(np.array([800.0]), 0.0)[0] == pytest.approx(800.0)
    b = H.BETA
    np.testing.assert_allclose(H.smooth_l1(np.array([0.0, b / 2, b, -1.0])),
                               [0.0, b / 8, b / 2, 1 - b / 2], rtol=1e-12)
    np.testing.assert_allclose(H.sigmoid(np.array([0.0, 50.0, -50.0])), [0.5, 1.0, np.exp(-50.0)], rtol=1e-12)


def test_adam_closed_form_for_constant_gradient():
    rng = np.random.default_rng(9)
    th = rng.standard_normal(10)
    g = rng.standard_normal(10)
    m = np.zeros(10)
    v = np.zeros(10)
    lr = 1e-2
    x = th.copy()
    for t in range(1, 6):
        # with a constant gradient the bias-corrected moments are g and g^2
        x, m, v = H.adam_step(x, g, m, v, t, lr)
        np.testing.assert_allclose(x, th - t * lr * g / (np.abs(g) + H.ADAM_EPS), rtol=1e-10, atol=1e-12)


def test_crop_and_stats_on_a_quadratic_surface():
    r = 5
    V = 2 * r + 1
    u0, v0, a, b = 2, 3, 0.01, 0.03
    yy, xx = np.mgrid[0:V, 0:V].astype(float)
    S = 1 - a * (yy - u0) ** 2 - b * (xx - v0) ** 2
    S[9, 9] = 0.8    # a planted second peak outside the exclusion
    crop, st = H.crop_and_stats(S, u0, v0, varT=4.0, varS=9.0, RT=2.0, mnz=16.0)
    assert crop[16, 16] == S[u0, v0] == 1.0
    inside = crop != -1.0
    assert inside.sum() == V * V          # the whole surface lies in the crop
    np.testing.assert_array_equal(crop[16 - u0:16 - u0 + V, 16 - v0:16 - v0 + V], S)
    # second best: the largest value outside the 3x3 block around the peak
    brute = max(S[y, x] for y in range(V) for x in range(V) if max(abs(y - u0), abs(x - v0)) > 1)
    assert st[1] == brute
    assert st[0] == 1.0 and st[2] == pytest.approx(S.mean()) and st[3] == pytest.approx(S.std())
    assert st[4] == pytest.approx(0.5) and st[5] == pytest.approx(0.75) and st[6] == pytest.approx(0.125)
    assert st[7] == pytest.approx(-(a + b))   # second differences of a quadratic: -2a, -2b


def test_features_statistics_match_direct_window_sums():
    rng = np.random.default_rng(10)
    img_r = rng.uniform(0, 1, (40, 44))
    img_s = np.roll(img_r, (1, -2), axis=(0, 1)) + 0.01 * rng.standard_normal((40, 44))
    p = O.Params(n_orient=2, s1=(1.0,), s2=(1.0,))
    Fr, Fs = O.sfoc(img_r, p), O.sfoc(img_s, p)
    m, r = 8, 3
    ips = np.array([[20, 20], [15, 25], [2, 2]], np.int32)
    prior = np.array([[0, 0], [-1, 1], [0, 0]], np.int32)
    cps, surf = O.match(Fs, Fr, ips, m, r, prior, want_surfaces=True)
    assert H.eligible(cps["flags"]).tolist() == [True, True, False]
    crops, stats = H.features(Fs, Fr, ips, prior, m, r, cps, surf)
    z = Fs.shape[2]
    mnz = m * m * z
    for i in range(len(ips)):
        if not H.eligible(cps["flags"][i:i + 1])[0]:
            assert not crops[i].any() and not stats[i].any()
            continue
        (ty, tx), (sy, sx) = O.window_origins(ips[i], prior[i], m, r)
        T = Fs[ty:ty + m, tx:tx + m]
        u, v = cps["dy"][i] + r, cps["dx"][i] + r
        Sw = Fr[sy + u:sy + u + m, sx + v:sx + v + m]
        assert stats[i, 4] == pytest.approx(T.std(), rel=1e-9)
        assert stats[i, 5] == pytest.approx(Sw.std(), rel=1e-7)
        assert stats[i, 6] == pytest.approx(T.mean(), rel=1e-12)
        assert stats[i, 0] == surf[i][u, v] == crops[i][16, 16]
    assert not H.eligible(cps["flags"][2:3])[0]   # out of bounds


def test_apply_decision():
    c = np.zeros(4, dtype=O.CP_DTYPE)
    c["flags"] = [O.VALID, O.INCONSISTENT, O.OOB, O.EDGE_PEAK]
    c["sub_dy"] = 0.3
    out = np.array([[2.0, 0.2, -3.0], [-1.0, 0.1, 0.1], [5.0, 1.0, 1.0], [5.0, 1.0, 1.0]])
    g = H.apply(c, out)
    assert g["flags"][0] == O.VALID | O.LEARNED and g["sub_dx"][0] == -1.5 and g["sub_dy"][0] == 0.2
    assert g["flags"][1] == O.INCONSISTENT | O.LEARNED
    assert g["flags"][2] == O.OOB and g["sub_dy"][2] == 0.3
    assert g["flags"][3] == O.EDGE_PEAK
