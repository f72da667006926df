"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these re-types an oracle formula: each compares it with an
independent route (finite differences of Eq. 1, rotated kernels, brute force,
library implementations, invariances, printed values)."""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import signal

from oracle import sfoc_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


# ------------------------------------------------------------- Eq. 1 -------
def test_gaussian_is_normalised_with_std_sigma():
    # Eq. 1 integrates to 1 and has second moment sigma^2: sigma is a
    # standard deviation (Section 2.1 reading), not a variance.
    for s in (0.6, 1.0, 2.5):
        h = 0.01
        x = np.arange(-12 * s, 12 * s + h, h)
        X, Y = np.meshgrid(x, x)
        g = O.gaussian(X, Y, s)
        assert abs(g.sum() * h * h - 1.0) < 1e-9
        assert abs((X * X * g).sum() * h * h - s * s) < 1e-6 * s * s


# ----------------------------------------------------------- Eq. 2-5 ------
@pytest.mark.parametrize("s", [0.6, 1.0, 1.5, 2.0, 3.0])
def test_basis_kernels_are_derivatives_of_eq1(s):
    k = O.basis_kernels(s)
    R = k["R"]
    y, x = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    G = lambda a, b: O.gaussian(a, b, s)
    h = 1e-4
    fdx = (G(x + h, y) - G(x - h, y)) / (2 * h)
    fdy = (G(x, y + h) - G(x, y - h)) / (2 * h)
    h2 = 1e-3
    fxx = (G(x + h2, y) - 2 * G(x, y) + G(x - h2, y)) / h2 ** 2
    fyy = (G(x, y + h2) - 2 * G(x, y) + G(x, y - h2)) / h2 ** 2
    fxy = (G(x + h2, y + h2) - G(x + h2, y - h2) - G(x - h2, y + h2) + G(x - h2, y - h2)) / (4 * h2 ** 2)
    scale = np.abs(k["gxx"]).max()
    assert np.abs(k["gx"] - fdx).max() < 1e-7 * scale
    assert np.abs(k["gy"] - fdy).max() < 1e-7 * scale
    for name, ref in (("gxx", fxx), ("gyy", fyy), ("gxy", fxy)):
        assert np.abs(k[name] - ref).max() < 1e-5 * scale, name


def test_kernel_support_and_antisymmetry():
    # Radius ceil(3 sigma); first-order kernels are exactly odd (so they sum
    # to zero) and second-order ones exactly even.
    for s, R in ((0.6, 2), (0.8, 3), (1.0, 3), (1.5, 5), (2.0, 6), (3.0, 9)):
        k = O.basis_kernels(s)
        assert k["R"] == R and k["gx"].shape == (2 * R + 1, 2 * R + 1)
        assert np.array_equal(k["gx"][:, ::-1], -k["gx"]) and np.array_equal(k["gy"][::-1], -k["gy"])
        assert np.array_equal(k["gxx"][::-1, ::-1], k["gxx"]) and np.array_equal(k["gxy"][:, ::-1], -k["gxy"])
        assert abs(k["gx"].sum()) < 1e-16 and abs(k["gxy"].sum()) < 1e-16


# ------------------------------------------------ steerability (Eq. 4-7) ---
def _directional_fd(s, theta, order, R):
    y, x = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    c, sn = math.cos(theta), math.sin(theta)
    G = lambda a, b: O.gaussian(a, b, s)
    if order == 1:
        h = 1e-4
        return (G(x + h * c, y + h * sn) - G(x - h * c, y - h * sn)) / (2 * h)
    h = 1e-3
    return (G(x + h * c, y + h * sn) - 2 * G(x, y) + G(x - h * c, y - h * sn)) / h ** 2


@pytest.mark.parametrize("theta", list(RNG.uniform(0, 2 * np.pi, 6)) + [k * np.pi / 8 for k in range(8)])
def test_steered_kernels_equal_rotated_derivative(theta):
    # A steerable filter is a combination of basis filters equal to the
    # rotated filter (Section 2.1, Eq. 4 and 7 read as directional derivatives).
    s = 1.7
    k = O.basis_kernels(s)
    (c, sn), (cc, ss, sc2) = O.steer_weights(theta)
    scale = np.abs(k["gxx"]).max()
    d1 = c * k["gx"] + sn * k["gy"]
    d2 = cc * k["gxx"] + ss * k["gyy"] + sc2 * k["gxy"]
    assert np.abs(d1 - _directional_fd(s, theta, 1, k["R"])).max() < 1e-7 * scale
    assert np.abs(d2 - _directional_fd(s, theta, 2, k["R"])).max() < 1e-5 * scale


def test_second_order_equals_freeman_adelson_interpolation():
    # k_j(theta) = (1 + 2 cos 2(theta - theta_j)) / 3 over 0, 60, 120 degrees
    # (Eq. 5) interpolates the true rotated second derivative exactly.
    s = 2.0
    k = O.basis_kernels(s)
    R = k["R"]
    for theta in RNG.uniform(0, np.pi, 5):
        acc = np.zeros((2 * R + 1, 2 * R + 1))
        for tj in (0.0, np.pi / 3, 2 * np.pi / 3):
            kj = (1 + 2 * math.cos(2 * (theta - tj))) / 3
            _, (cc, ss, sc2) = O.steer_weights(tj)
            acc += kj * (cc * k["gxx"] + ss * k["gyy"] + sc2 * k["gxy"])
        _, (cc, ss, sc2) = O.steer_weights(theta)
        d2 = cc * k["gxx"] + ss * k["gyy"] + sc2 * k["gxy"]
        assert np.abs(acc - d2).max() < 1e-15


def test_literal_eq7_bases_are_not_steerable():
    # Documents the reading: the printed G2^60 = Gyy - Gxy, G2^120 = Gyy + Gxy
    # with weights cos^2, sin^2, -2 sin cos do not give a rotated filter.
    s = 2.0
    k = O.basis_kernels(s)
    theta = 0.7
    c, sn = math.cos(theta), math.sin(theta)
    lit = c * c * k["gxx"] + sn * sn * (k["gyy"] - k["gxy"]) - 2 * sn * c * (k["gyy"] + k["gxy"])
    d2 = _directional_fd(s, theta, 2, k["R"])
    assert np.abs(lit - d2).max() > 0.1 * np.abs(d2).max()


# ------------------------------------------------------- plumbing pins -----
def test_reflect101_matches_numpy_reflect():
    def np_ext(a, pad):
        for ax in (0, 1):
            w = [(0, 0), (0, 0)]
            w[ax] = (pad, pad)
            a = np.pad(a, w, mode="edge" if a.shape[ax] == 1 else "reflect")
        return a
    for n in (1, 2, 5, 13):
        a = RNG.standard_normal((n, n + 1))
        for pad in (0, 1, 3, 2 * n + 3):
            assert np.array_equal(O.extend(a, pad), np_ext(a, pad))


def test_conv2d_valid_matches_scipy():
    E = RNG.standard_normal((30, 27))
    k = RNG.standard_normal((7, 7))
    assert np.allclose(O.conv2d_valid(E, k), signal.convolve2d(E, k, mode="valid"), atol=1e-12)


# -------------------------------------------------------- SFOC pins --------
def _img(h=40, w=40, seed=0):
    from paper_2202_13347_amd import synth
    return synth.make_pair(seed, (h, w), 2.0).ref.astype(np.float64)


def test_sfoc_steered_channel_equals_rotated_kernel_convolution():
    # Channel k (signed, one scale, before smoothing) is the image convolved
    # with the directly rotated derivative kernel at theta_k = k pi / N.
    img = _img(36, 33)
    p = O.Params(n_orient=6, s1=(1.5,), s2=(1.5,), rectify="signed")
    A, Q = O.sfoc_unnormalised(img, p)
    R = O.radius(1.5, 3.0)
    E = O.extend(img, R + Q)
    for kk in range(6):
        th = kk * np.pi / 6
        for order in (1, 2):
            ref = signal.convolve2d(E, _directional_fd(1.5, th, order, R), mode="valid")
            got = A[kk + (order - 1) * 6]
            assert np.abs(got - ref).max() < (1e-6 if order == 1 else 1e-4) * np.abs(ref).max()


def test_sfoc_rot90_permutes_channels():
    # Rotating the image by 90 degrees turns direction theta into theta +- pi/2,
    # i.e. channel k -> k + N/2 (mod N) in each order block.
    img = _img(30, 30, 3)
    p = O.Params()
    F = O.sfoc(img, p)
    Fr = O.sfoc(np.rot90(img), p)
    N = p.n_orient
    perm = [(k + N // 2) % N for k in range(N)]
    perm = perm + [N + q for q in perm]
    # rot90 (counter-clockwise) of the channel maps, channels permuted.
    got = np.rot90(F, axes=(0, 1))
    # Match each rotated channel against the permuted one (direction choice only
    # decides the sign of the shift; accept either).
    perm2 = [(k - N // 2) % N for k in range(N)]
    perm2 = perm2 + [N + q for q in perm2]
    e1 = np.abs(Fr[:, :, perm] - got).max()
    e2 = np.abs(Fr[:, :, perm2] - got).max()
    assert min(e1, e2) < 1e-12


def test_sfoc_transpose_maps_theta_to_half_pi_minus_theta():
    img = _img(26, 31, 4)
    p = O.Params()
    F = O.sfoc(img, p)
    Ft = O.sfoc(img.T, p)
    N = p.n_orient
    perm = [(N // 2 - k) % N for k in range(N)]
    perm = perm + [N + q for q in perm]
    assert np.abs(Ft[:, :, perm] - F.transpose(1, 0, 2)).max() < 1e-12


def test_sfoc_contrast_and_scale_invariance():
    img = _img(28, 28, 5)
    p = O.Params(eps=0.0)
    F = O.sfoc(img, p)
    assert np.abs(O.sfoc(-img, p) - F).max() < 1e-12          # |.| rectification
    assert np.abs(O.sfoc(3.7 * img, p) - F).max() < 1e-12     # L2 normalisation
    # First-order channels are offset invariant (derivative kernels sum to 0).
    Fo = O.sfoc(img + 5.0, p)
    assert np.abs(Fo[:, :, :8] - F[:, :, :8]).max() < 1e-9


def test_sfoc_normalisation_gives_unit_norm_per_order():
    img = _img(24, 24, 6)
    F = O.sfoc(img, O.Params(eps=0.0))
    n1 = (F[:, :, :8] ** 2).sum(axis=2)
    n2 = (F[:, :, 8:] ** 2).sum(axis=2)
    assert np.abs(n1 - 1).max() < 1e-14 and np.abs(n2 - 1).max() < 1e-14
    assert np.abs((F ** 2).sum(axis=2) - 2.0).max() < 1e-14
    assert F.min() >= 0.0


def test_dilated_smoothing_impulse_response():
    # Three 3x3 Gaussians with holes at rates 1, 2, 3, summed (Section 2.1).
    H = W = 15
    Q = 3
    A = np.zeros((H + 2 * Q, W + 2 * Q))
    A[Q + 7, Q + 7] = 1.0
    sd = 1.3
    out = O.dilated_smooth(A, Q, H, W, sd, 1, (1, 2, 3))
    # Response at p is sum over taps hitting the impulse: support = {7 - r*i}.
    nz = set(zip(*np.nonzero(out)))
    expect = {(7 - r * i, 7 - r * j) for r in (1, 2, 3) for i in (-1, 0, 1) for j in (-1, 0, 1)}
    assert nz == expect
    assert abs(out.sum() - 3.0) < 1e-14
    w1 = math.exp(-1 / (2 * sd * sd))
    w0n = 1 / (1 + 2 * w1)
    assert abs(out[7, 7] - 3 * w0n ** 2) < 1e-15
    assert abs(out[7, 9] - w0n * w0n * w1) < 1e-15   # rate 2 edge tap


def test_sfoc_border_is_reflect101_of_input_only():
    # Every stage is evaluated on the extended input: SFOC of an image equals
    # the centre crop of SFOC of its (larger) reflect-101 extension.
    img = _img(22, 19, 7)
    p = O.Params()
    P = 9 + 3 + 2
    F = O.sfoc(img, p)
    Fb = O.sfoc(O.extend(img, P), p)
    assert np.abs(Fb[P:P + 22, P:P + 19] - F).max() < 1e-12


def test_sfoc_paper_preset_and_first_order_only():
    img = _img(20, 20, 8)
    pp = O.preset_paper()
    assert pp.z == 12 and O.sfoc(img, pp).shape == (20, 20, 12)
    f = O.Params(second_order=False)
    Ff = O.sfoc(img, f)
    assert Ff.shape == (20, 20, 8)
    assert np.abs(Ff - O.sfoc(img, O.Params())[:, :, :8]).max() < 1e-13


# ----------------------------------------------- integral images (Eq. 14-16)
def test_integral_image_box_sums_exact_on_integers():
    g = RNG.integers(-50, 50, size=(9, 11)).astype(np.float64)
    G = O.integral_image(g)
    for y in range(9):
        for x in range(11):
            for m in range(1, 10 - y):
                for n in range(1, 12 - x):
                    assert O.box_sum(G, y, x, m, n) == g[y:y + m, x:x + n].sum()


def test_integral_feature_images_sum_over_channels():
    F = RNG.integers(0, 9, size=(6, 7, 4)).astype(np.float64)
    G1, G2 = O.integral_feature_images(F)
    assert O.box_sum(G1, 1, 2, 3, 4) == F[1:4, 2:6, :].sum()
    assert O.box_sum(G2, 0, 0, 6, 7) == (F * F).sum()


# ----------------------------------------------------- NCC (Eq. 8-13) ------
def test_fft_correlation_matches_direct_sum():
    S = RNG.standard_normal((11, 12, 3))
    T = RNG.standard_normal((4, 5, 3))
    R = O.correlate_fft(S, T)
    for u in range(8):
        for v in range(8):
            assert abs(R[u, v] - (S[u:u + 4, v:v + 5] * T).sum()) < 1e-12


@settings(max_examples=40, deadline=None)
@given(m=st.integers(3, 8), r=st.integers(1, 4), z=st.integers(1, 16), seed=st.integers(0, 2 ** 31))
def test_fast_ncc_equals_bruteforce_eq8(m, r, z, seed):
    rng = np.random.default_rng(seed)
    M = m + 2 * r
    S = rng.uniform(0, 1, (M, M, z))
    T = rng.uniform(0, 1, (m, m, z))
    a, flat_a = O.ncc_bruteforce(S, T)
    b, flat_b, nf = O.ncc_fast(S, T)
    assert flat_a == flat_b and not nf
    assert np.abs(a - b).max() < 1e-10


def test_ncc_is_one_at_planted_offset_and_bounded():
    S = RNG.uniform(0, 1, (20, 20, 5))
    T = S[7:15, 3:11].copy()
    a, _ = O.ncc_bruteforce(S, T)
    b, _, _ = O.ncc_fast(S, T)
    for ncc in (a, b):
        assert abs(ncc[7, 3] - 1.0) < 1e-12
        assert np.unravel_index(np.argmax(ncc), ncc.shape) == (7, 3)
        assert np.abs(ncc).max() <= 1 + 1e-12


def test_ncc_affine_intensity_invariance():
    S = RNG.uniform(0, 1, (16, 16, 4))
    T = RNG.uniform(0, 1, (6, 6, 4))
    base, _, _ = O.ncc_fast(S, T)
    for a, b in ((2.5, -1.0), (0.3, 4.0)):
        assert np.abs(O.ncc_fast(a * S + b, T)[0] - base).max() < 1e-11
        assert np.abs(O.ncc_fast(S, a * T + b)[0] - base).max() < 1e-11
    assert np.abs(O.ncc_fast(-2.0 * S + 1, T)[0] + base).max() < 1e-11


def test_flat_template_and_flat_positions():
    S = RNG.uniform(0, 1, (10, 10, 2))
    T = np.full((4, 4, 2), 0.3)
    _, flat = O.ncc_bruteforce(S, T)
    assert flat and O.ncc_fast(S, T)[1]
    S2 = S.copy(); S2[:5, :5] = 0.7
    T2 = RNG.uniform(0, 1, (4, 4, 2))
    a, _ = O.ncc_bruteforce(S2, T2)
    b, _, _ = O.ncc_fast(S2, T2)
    assert a[0, 0] == 0.0 and b[0, 0] == 0.0 and a[1, 1] == 0.0


# ------------------------------------------------------- peak / CP ---------
def test_parabola_exact_on_quadratics():
    for t0 in (-0.45, -0.1, 0.0, 0.2, 0.49):
        a, b = -2.3, 0.8
        c = [a * (t - t0) ** 2 + b for t in (-1, 0, 1)]
        assert abs(O.parabola_offset(*c) - t0) < 1e-14
    assert O.parabola_offset(1.0, 1.0, 1.0) == 0.0
    assert O.parabola_offset(0.0, 1.0, 1.0) == 0.5      # clamped


def test_argmax_ties_take_smallest_row_major_index():
    s = np.zeros((5, 5)); s[2, 3] = 1.0; s[3, 1] = 1.0; s[2, 4] = 1.0
    u, v, sc, su, sv, edge = O.peak(s)
    assert (u, v) == (2, 3) and sc == 1.0 and not edge
    s2 = np.zeros((5, 5)); s2[0, 2] = 1
    assert O.peak(s2)[5]


def test_exact_recovery_of_integer_shifts():
    # Noise-free same-modality pair with integer shift d: sen(p) = ref(p + d),
    # IPs far enough from the borders that SFOC supports lie inside both.
    rng = np.random.default_rng(77)
    from paper_2202_13347_amd import synth
    canvas = synth.make_pair(11, 160, 1.0, noise_std=0.0).ref.astype(np.float64)
    p = O.Params()
    m, r = 16, 6
    for trial in range(3):
        d = rng.integers(-5, 6, size=2)
        o = 16
        ref = canvas[o:o + 120, o:o + 120]
        sen = canvas[o + d[0]:o + d[0] + 120, o + d[1]:o + d[1] + 120]
        ips = np.array([[40, 40], [60, 75], [80, 50]])
        cps, surf = O.register_cps(ref, sen, ips, m, r, p, want_surfaces=True)
        assert np.all(cps["dy"] == d[0]) and np.all(cps["dx"] == d[1])
        assert np.all(np.abs(cps["score"] - 1.0) < 1e-12)
        assert np.all(np.abs(cps["sub_dy"]) < 0.1) and np.all(np.abs(cps["sub_dx"]) < 0.1)
        assert np.all(cps["flags"] == O.VALID)
        b, _ = O.match(O.sfoc(sen, p), O.sfoc(ref, p), ips, m, r, method="brute", want_surfaces=True)
        assert np.array_equal(b["dy"], cps["dy"]) and np.array_equal(b["dx"], cps["dx"])


def test_oob_and_prior():
    F = RNG.uniform(0, 1, (40, 40, 2))
    cps = O.match(F, F, np.array([[3, 20], [20, 20]]), 8, 3)
    assert cps["flags"][0] == O.OOB and cps["dy"][1] == 0 and cps["dx"][1] == 0
    # prior shifts the search window: the template found at prior + d.
    Fr = np.roll(F, (2, -3), axis=(0, 1))
    cps = O.match(F, Fr, np.array([[20, 20]]), 8, 2, prior=np.array([[2, -2]]))
    assert (cps["dy"][0], cps["dx"][0]) == (0, -1)


def test_consistency_flags_outliers():
    cps = np.zeros(7, dtype=O.CP_DTYPE)
    cps["dy"] = [3, 3, 3, 4, 3, 9, 3]
    cps["dx"] = [-1, -1, -2, -1, -1, -1, -1]
    cps["sub_dy"] = [0.1, -0.1, 0.0, 0.4, 0.2, 0.0, 0.0]
    cps["flags"][6] = O.EDGE_PEAK
    O.consistency(cps)
    assert list(cps["flags"]) == [1, 1, 1, 1, 1, O.INCONSISTENT, O.EDGE_PEAK]


# ------------------------------------------------ quantisation -----------
def test_bf16_and_f16_rounding_match_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([RNG.standard_normal(5000).astype(np.float32),
                        np.array([1.00390625, 1.01171875, -3.0e-39, 65504.0, 1e5], np.float32)])
    tb = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(O.round_to_bf16(x), tb)
    th = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(O.round_to_f16(x), th)


# ------------------------------------------------ Eq. 17-19 (golden) -------
def test_cost_model_worked_example():
    with open(os.path.join(GOLD, "eq19_worked_example.json")) as f:
        g = json.load(f)
    got = 100.0 * O.cost_ratio(g["m"], g["M"], g["z"])
    assert round(got, 3) == g["ratio_percent"]


def test_region_oracle_equals_dense_crop():
    # The crop-with-halo evaluation reproduces the dense descriptor exactly,
    # at borders too (reflect-101 of the whole image).
    img = _img(41, 37, 9)
    p = O.Params()
    F = O.sfoc(img, p)
    for (y0, x0, h, w) in ((0, 0, 10, 12), (30, 25, 11, 12), (5, 17, 20, 9), (35, 0, 6, 37)):
        assert np.abs(O.sfoc_region(img, y0, x0, h, w, p) - F[y0:y0 + h, x0:x0 + w]).max() < 1e-13


def test_region_match_equals_dense_match():
    from paper_2202_13347_amd import synth
    pr = synth.make_pair(3, 96, 4.0)
    p = O.Params()
    ips = np.array([[30, 30], [48, 60], [65, 40], [5, 5]])
    cps, surf = O.register_cps(pr.ref, pr.sen, ips, 16, 6, p, want_surfaces=True)
    for i, ip in enumerate(ips):
        rec, s = O.match_one_region(pr.ref, pr.sen, ip, 16, 6, p)
        assert rec[0] == cps["dy"][i] and rec[1] == cps["dx"][i]
        assert rec[5] == (int(cps["flags"][i]) & ~(O.VALID | O.INCONSISTENT))
        assert np.abs(s - surf[i]).max() < 1e-10


def test_region_variants_equal_dense_match_per_rounding():
    # The several-roundings crop evaluation gives, for each rounding, the
    # dense oracle's CP on descriptors rounded the same way.
    from paper_2202_13347_amd import synth
    pr = synth.make_pair(4, 96, 4.0)
    p = O.Params()
    ips = np.array([[30, 30], [48, 60], [65, 40], [5, 5]])
    kinds = (None, "bf16", "f16")
    dense = {k: O.register_cps(pr.ref, pr.sen, ips, 16, 6, p, quantise=k, want_surfaces=True) for k in kinds}
    for i, ip in enumerate(ips):
        res = O.match_one_region_variants(pr.ref, pr.sen, ip, 16, 6, p, quantise=kinds)
        assert len(res) == 3
        for k, (rec, s) in zip(kinds, res):
            cps, surf = dense[k]
            assert rec[0] == cps["dy"][i] and rec[1] == cps["dx"][i]
            assert rec[5] == (int(cps["flags"][i]) & ~(O.VALID | O.INCONSISTENT))
            assert np.abs(s - surf[i]).max() < 1e-10
    # rounding changes the surfaces (the variants are not the same computation)
    r0 = O.match_one_region_variants(pr.ref, pr.sen, ips[0], 16, 6, p, quantise=kinds)
    assert np.abs(r0[0][1] - r0[1][1]).max() > 1e-6
