"""Plain FP64 CPU reference ("the oracle") for dense SFOC descriptors and
Fast-NCC_SFOC template matching (Ye et al., arXiv 2202.13347, Sections 2.1,
2.2 and 3.2.2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call this module.  The GPU
library never uses it, shares no code with it, and must fail loudly rather
than fall back to it.

Everything is computed in float64 with NumPy, in the order the paper states
the method and with no blocking or fusion: the 2-D kernels are sampled from
their closed forms (Eq. 1-3, 5), convolved with the image one scale at a
time, steered per scale and then summed over scales (Eq. 6, 7), rectified,
smoothed with the three dilated Gaussian kernels (Section 2.1), normalised
per order and stacked.  NCC is given both by its definition (Eq. 8, brute
force) and by the fast form (Eq. 9-16: an FFT cross-correlation plus
integral images).

Readings of passages that are garbled or silent in the paper (each is listed
with its justification in the design notes shipped with the repository):
  * sigma is a standard deviation (the paper calls it both).
  * Second-order steering uses the directional second derivative
    cos^2 Gxx + 2 sin cos Gxy + sin^2 Gyy in (x = column, y = row) axes, the
    reading of Eq. 7 under which the filter is steerable; the printed Eq. 5/7
    bases are not (see steering pins in the tests).
  * Kernel support is [-R, R]^2 with R = ceil(trunc * sigma), point sampled.
  * The input image is extended by reflect-101 and every stage is evaluated
    on the extended domain, then cropped.
  * Responses are rectified with |.| after the sum over scales.
  * Dilated smoothing: 3x3 Gaussian base (K = 1) at rates 1, 2, 3, summed;
    sigma_d = sd1 for first-order channels, sd2 for second-order ones.
  * Normalisation: per-pixel L2 within each order block, eps under the root.
  * NCC uses one mean over all m*n*z entries (Eq. 8/9); positions whose
    search variance is <= tau get NCC 0; tau = 1e-12 * m*n*z.
  * CP = argmax (ties -> smallest row-major index), separable three-point
    parabola for the sub-pixel part, and a median-translation consistency
    check at the paper's 1.5 px correctness threshold (Section 4.1).

Parity status: the SFOC constants that the paper does not give (the dilated
base sigma_d values, the base kernel size, eps) are "parity unpinned" against
the paper; every other function is pinned by the CPU tests against closed
forms, invariances, brute force and printed values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CP flags (bit values shared with the C header by value, not by code).
VALID, OOB, FLAT_T, FLAT_S, EDGE_PEAK, INCONSISTENT, LEARNED, NONFINITE = (
    1, 2, 4, 8, 16, 32, 64, 128)
CONSISTENCY_PX = 1.5  # Section 4.1: a match within 1.5 px is correct.

CP_DTYPE = np.dtype([("sen_row", np.int32), ("sen_col", np.int32),
                     ("dy", np.int32), ("dx", np.int32),
                     ("sub_dy", np.float64), ("sub_dx", np.float64),
                     ("score", np.float64), ("flags", np.uint32)])


@dataclass
class Params:
    """SFOC parameters.  n_orient orientations k*pi/N (Section 2.1 uses 6);
    s1 / s2: Gaussian standard deviations of the first- / second-order
    channels, summed over (Section 2.1, Table 2)."""
    n_orient: int = 8
    s1: tuple = (1.0, 2.0, 3.0)
    s2: tuple = (1.0, 2.0, 3.0)
    trunc: float = 3.0
    sd1: float = 1.0
    sd2: float = 1.5
    K: int = 1
    dil: tuple = (1, 2, 3)
    eps: float = 1e-8
    rectify: str = "abs"          # "abs" | "signed" | "relu"
    second_order: bool = True     # False -> F-SFOC (first-order channels only)

    @property
    def z(self) -> int:
        return self.n_orient * (2 if self.second_order else 1)


def preset_paper() -> Params:
    """Section 2.1 (six directions) and Table 2 (sigma 0.6/0.8/1.0; 1.5)."""
    return Params(n_orient=6, s1=(0.6, 0.8, 1.0), s2=(1.5,))


def preset_baseline() -> Params:
    """Eight orientations, sigma = 1, 2, 3 for both orders."""
    return Params()


def radius(sigma: float, trunc: float) -> int:
    return int(math.ceil(trunc * sigma - 1e-9))


# ---------------------------------------------------------------- Eq. 1-5 --
def gaussian(x, y, s):
    """Eq. 1: 2-D Gaussian with standard deviation s."""
    return np.exp(-(x * x + y * y) / (2.0 * s * s)) / (2.0 * np.pi * s * s)


def basis_kernels(s: float, trunc: float = 3.0) -> dict:
    """Eq. 2, 3 and 5 sampled on the integer grid [-R, R]^2.

    Arrays are indexed [dy + R, dx + R]; x is the column offset and y the row
    offset (rows grow downwards)."""
    R = radius(s, trunc)
    y, x = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    e = np.exp(-(x * x + y * y) / (2.0 * s * s))
    c4 = 1.0 / (2.0 * np.pi * s ** 4)
    return {
        "R": R,
        "gx": -c4 * x * e,                                   # Eq. 2
        "gy": -c4 * y * e,                                   # Eq. 3
        "gxx": -c4 * (1.0 - x * x / (s * s)) * e,            # Eq. 5
        "gyy": -c4 * (1.0 - y * y / (s * s)) * e,            # Eq. 5
        "gxy": (x * y / (2.0 * np.pi * s ** 6)) * e,         # Eq. 5
    }


def steer_weights(theta: float):
    """Eq. 4 / 6 and the steerable reading of Eq. 7 for direction theta."""
    c, s = math.cos(theta), math.sin(theta)
    return (c, s), (c * c, s * s, 2.0 * s * c)   # (gx, gy), (gxx, gyy, gxy)


def orientations(n: int):
    """Section 2.1: directions k*pi/n, k = 0..n-1, over [0, pi)."""
    return [k * math.pi / n for k in range(n)]


# ------------------------------------------------------------ plumbing ----
def reflect101_index(i: np.ndarray, n: int) -> np.ndarray:
    """Reflect-101 (mirror without repeating the edge), periodic for any i."""
    i = np.asarray(i)
    if n == 1:
        return np.zeros_like(i)
    p = 2 * (n - 1)
    j = np.mod(i, p)
    return np.where(j > n - 1, p - j, j)


def extend(img: np.ndarray, pad: int) -> np.ndarray:
    H, W = img.shape
    ry = reflect101_index(np.arange(-pad, H + pad), H)
    rx = reflect101_index(np.arange(-pad, W + pad), W)
    return img[np.ix_(ry, rx)]


def conv2d_valid(E: np.ndarray, k: np.ndarray) -> np.ndarray:
    """True 2-D convolution (out[p] = sum_q k[q] E[p - q]) at the positions
    where the whole kernel lies inside E."""
    R = k.shape[0] // 2
    OH, OW = E.shape[0] - 2 * R, E.shape[1] - 2 * R
    out = np.zeros((OH, OW))
    for a in range(2 * R + 1):
        dy = a - R
        for b in range(2 * R + 1):
            dx = b - R
            w = k[a, b]
            if w != 0.0:
                out += w * E[R - dy:R - dy + OH, R - dx:R - dx + OW]
    return out


def dilated_weights(sd: float, K: int) -> np.ndarray:
    w = np.exp(-np.arange(-K, K + 1) ** 2 / (2.0 * sd * sd))
    return w / w.sum()


# -------------------------------------------------------------- SFOC -------
def halo(p: Params) -> int:
    """Reach of one output pixel into the input: largest radius + K*max(dil)."""
    sig_all = list(p.s1) + (list(p.s2) if p.second_order else [])
    return max(radius(s, p.trunc) for s in sig_all) + p.K * max(p.dil)


def steered_valid(crop: np.ndarray, p: Params):
    """Steered (Eq. 4/6, 7), scale-summed, rectified channels of `crop`,
    evaluated where the whole support lies inside it.  For a crop carrying a
    halo of P = halo(p) around an H x W region, returns (A, Q) with
    A: (z, H+2Q, W+2Q) on the region grown by Q = K*max(dil)."""
    crop = np.asarray(crop, dtype=np.float64)
    P = halo(p)
    Q = p.K * max(p.dil)
    H, W = crop.shape[0] - 2 * P, crop.shape[1] - 2 * P
    thetas = orientations(p.n_orient)

    def region(R):
        o = P - Q - R
        return crop[o:o + H + 2 * Q + 2 * R, o:o + W + 2 * Q + 2 * R]

    A = []
    F1 = [np.zeros((H + 2 * Q, W + 2 * Q)) for _ in thetas]
    for s in p.s1:                                   # one scale at a time
        k = basis_kernels(s, p.trunc)
        Ereg = region(k["R"])
        bx, by = conv2d_valid(Ereg, k["gx"]), conv2d_valid(Ereg, k["gy"])   # Eq. 6
        for i, th in enumerate(thetas):
            (c, sn), _ = steer_weights(th)
            F1[i] += c * bx + sn * by                # summed over scales
    A.extend(F1)
    if p.second_order:
        F2 = [np.zeros((H + 2 * Q, W + 2 * Q)) for _ in thetas]
        for s in p.s2:
            k = basis_kernels(s, p.trunc)
            Ereg = region(k["R"])
            bxx, byy, bxy = (conv2d_valid(Ereg, k[n]) for n in ("gxx", "gyy", "gxy"))  # Eq. 7
            for i, th in enumerate(thetas):
                _, (cc, ss, sc2) = steer_weights(th)
                F2[i] += cc * bxx + ss * byy + sc2 * bxy
        A.extend(F2)
    A = np.stack(A)
    if p.rectify == "abs":
        A = np.abs(A)
    elif p.rectify == "relu":
        A = np.maximum(A, 0.0)
    elif p.rectify != "signed":
        raise ValueError(p.rectify)
    return A, Q


def sfoc_unnormalised(img: np.ndarray, p: Params):
    """steered_valid over the reflect-101 extended image: (A, Q)."""
    return steered_valid(extend(np.asarray(img, dtype=np.float64), halo(p)), p)


def dilated_smooth(A: np.ndarray, Q: int, H: int, W: int, sd: float, K: int, dil) -> np.ndarray:
    """Sum over rates r of the (2K+1)^2 Gaussian with holes at r (Section 2.1,
    Fig. 3), evaluated at the H x W positions of a map given on the domain
    extended by Q."""
    w = dilated_weights(sd, K)
    out = np.zeros((H, W))
    for r in dil:
        for i in range(-K, K + 1):
            for j in range(-K, K + 1):
                out += w[i + K] * w[j + K] * A[Q + r * i:Q + r * i + H, Q + r * j:Q + r * j + W]
    return out


def sfoc_valid(crop: np.ndarray, p: Params) -> np.ndarray:
    """All SFOC stages on a crop that carries a halo of P = halo(p): the
    (H, W, z) descriptor of its centre, channels [first-order k = 0..N-1,
    second-order k = 0..N-1]."""
    A, Q = steered_valid(crop, p)
    H, W = A.shape[1] - 2 * Q, A.shape[2] - 2 * Q
    N = p.n_orient
    D = np.stack([dilated_smooth(A[c], Q, H, W, p.sd1 if c < N else p.sd2, p.K, p.dil)
                  for c in range(A.shape[0])])
    out = np.empty_like(D)
    for lo in range(0, D.shape[0], N):
        blk = D[lo:lo + N]
        out[lo:lo + N] = blk / np.sqrt((blk * blk).sum(axis=0) + p.eps)   # per order
    return np.ascontiguousarray(out.transpose(1, 2, 0))


def sfoc(img: np.ndarray, p: Params | None = None) -> np.ndarray:
    """Dense SFOC descriptor (H, W, z) float64 of an image: every stage is
    evaluated on the reflect-101 extended image, then cropped."""
    p = p or Params()
    return sfoc_valid(extend(np.asarray(img, dtype=np.float64), halo(p)), p)


def sfoc_region(img: np.ndarray, y0: int, x0: int, h: int, w: int, p: Params | None = None) -> np.ndarray:
    """Rows y0..y0+h-1, columns x0..x0+w-1 of sfoc(img), from a crop of the
    extended image (each output pixel sees exactly the values the dense
    evaluation sees).  (h, w, z)."""
    p = p or Params()
    P = halo(p)
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    ry = reflect101_index(np.arange(y0 - P, y0 + h + P), H)
    rx = reflect101_index(np.arange(x0 - P, x0 + w + P), W)
    return sfoc_valid(img[np.ix_(ry, rx)], p)


# -------------------------------------------------------- rounding ---------
def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even), returned as
    float32 holding the rounded value.  Non-finite values pass through."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = r.astype(np.uint32)
    out = r.view(np.float32).copy()
    bad = ~np.isfinite(f)
    out[bad] = f[bad]
    return out


def round_to_f16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to IEEE binary16 (NumPy's cast is round to nearest
    even), returned as float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


# ----------------------------------------------------- integral images -----
def integral_image(g2d: np.ndarray) -> np.ndarray:
    """Eq. 15: single-pass recursion s(x,y) = s(x,y-1) + g(x,y),
    G(x,y) = G(x-1,y) + s(x,y), stored with a zero first row and column, so
    G[y, x] is the sum of g over rows < y and columns < x."""
    H, W = g2d.shape
    G = np.zeros((H + 1, W + 1))
    s = np.cumsum(np.asarray(g2d, dtype=np.float64), axis=1)   # running column sum
    G[1:, 1:] = np.cumsum(s, axis=0)
    return G


def integral_feature_images(F: np.ndarray):
    """Eq. 14 over channels: integral images of sum_h g and sum_h g^2."""
    F = np.asarray(F, dtype=np.float64)
    return integral_image(F.sum(axis=2)), integral_image((F * F).sum(axis=2))


def box_sum(G: np.ndarray, y, x, m: int, n: int):
    """Eq. 16: sum over rows y..y+m-1 and columns x..x+n-1 by four lookups."""
    return G[y + m, x + n] - G[y, x + n] - G[y + m, x] + G[y, x]


# ---------------------------------------------------------- matching -------
def window_origins(ip, prior, m: int, r: int):
    """Template origin (rows p - floor(m/2) ...) and search-window origin
    (template origin - r + prior)."""
    ty, tx = int(ip[0]) - m // 2, int(ip[1]) - m // 2
    py, px = (0, 0) if prior is None else (int(prior[0]), int(prior[1]))
    return (ty, tx), (ty - r + py, tx - r + px)


def in_bounds(y, x, h, w, H, W):
    return y >= 0 and x >= 0 and y + h <= H and x + w <= W


def ncc_bruteforce(S: np.ndarray, T: np.ndarray):
    """Eq. 8 evaluated directly at every valid position of T inside S.

    S: (M, M', z), T: (m, n, z).  Returns (ncc, flatT) with ncc of shape
    (M-m+1, M'-n+1); positions whose search variance is <= tau give 0."""
    S = np.asarray(S, np.float64); T = np.asarray(T, np.float64)
    m, n, z = T.shape
    mnz = m * n * z
    tau = 1e-12 * mnz
    dT = T - T.mean()
    varT = (dT * dT).sum()
    Vy, Vx = S.shape[0] - m + 1, S.shape[1] - n + 1
    out = np.zeros((Vy, Vx))
    flatT = not (varT > tau)
    if flatT:
        return out, True
    for u in range(Vy):
        for v in range(Vx):
            w = S[u:u + m, v:v + n, :]
            dS = w - w.mean()
            varS = (dS * dS).sum()
            if varS > tau:
                out[u, v] = (dS * dT).sum() / math.sqrt(varS * varT)
    return out, False


def correlate_fft(S: np.ndarray, T: np.ndarray, L: int | None = None) -> np.ndarray:
    """Eq. 10 / 13: R_ST(u, v) = sum_h sum_ij S(u+i, v+j, h) T(i, j, h) as
    IFFT[ sum_h FFT(S_h) conj(FFT(T_h)) ] on an L x L grid (L >= M avoids
    wrap-around on the valid region)."""
    M, Mx, z = S.shape
    m, n, _ = T.shape
    Ly = L or M
    Lx = L or Mx
    acc = np.zeros((Ly, Lx), dtype=np.complex128)
    for h in range(z):
        acc += np.fft.fft2(S[:, :, h], s=(Ly, Lx)) * np.conj(np.fft.fft2(T[:, :, h], s=(Ly, Lx)))
    R = np.fft.ifft2(acc).real
    return R[:M - m + 1, :Mx - n + 1]


def ncc_fast(S: np.ndarray, T: np.ndarray, G1=None, G2=None, origin=(0, 0)):
    """Eq. 9-16: NCC from the FFT correlation and integral images.

    G1, G2: integral images of sum_h g and sum_h g^2 of the image S was cut
    from, with `origin` the window's top-left in that image; if None they are
    built over the window itself.  Returns (ncc, flatT, nonfinite)."""
    S = np.asarray(S, np.float64); T = np.asarray(T, np.float64)
    m, n, z = T.shape
    mnz = float(m * n * z)
    tau = 1e-12 * mnz
    if G1 is None:
        G1, G2 = integral_feature_images(S)
        origin = (0, 0)
    RT = T.sum(); RTT = (T * T).sum()                 # Eq. 12
    varT = RTT - RT * RT / mnz
    Vy, Vx = S.shape[0] - m + 1, S.shape[1] - n + 1
    if not (np.isfinite(RT) and np.isfinite(RTT)):
        return np.zeros((Vy, Vx)), False, True
    if not (varT > tau):
        return np.zeros((Vy, Vx)), True, False
    RST = correlate_fft(S, T)                           # Eq. 13
    u = np.arange(Vy)[:, None] + origin[0]
    v = np.arange(Vx)[None, :] + origin[1]
    RS = box_sum(G1, u, v, m, n)                        # Eq. 11 via Eq. 16
    RSS = box_sum(G2, u, v, m, n)
    varS = RSS - RS * RS / mnz
    nonfinite = not (np.all(np.isfinite(RST)) and np.all(np.isfinite(varS)) and np.all(np.isfinite(RS)))
    num = RST - RS * RT / mnz                           # Eq. 9
    with np.errstate(invalid="ignore", divide="ignore"):
        ncc = np.where(varS > tau, num / np.sqrt(np.maximum(varS, 0.0) * varT), 0.0)
    return ncc, False, nonfinite


def parabola_offset(cm: float, c0: float, cp: float) -> float:
    """Vertex of the parabola through (-1, cm), (0, c0), (1, cp)."""
    den = cm - 2.0 * c0 + cp
    if not den < 0.0:
        return 0.0
    d = (cm - cp) / (2.0 * den)
    return float(min(0.5, max(-0.5, d)))


def peak(ncc: np.ndarray):
    """Argmax (ties -> smallest row-major index) and separable parabola fit.
    Returns (u, v, score, sub_u, sub_v, edge)."""
    idx = int(np.argmax(ncc))            # NumPy returns the first maximum
    Vy, Vx = ncc.shape
    u, v = divmod(idx, Vx)
    edge = u == 0 or v == 0 or u == Vy - 1 or v == Vx - 1
    su = sv = 0.0
    if not edge:
        su = parabola_offset(ncc[u - 1, v], ncc[u, v], ncc[u + 1, v])
        sv = parabola_offset(ncc[u, v - 1], ncc[u, v], ncc[u, v + 1])
    return u, v, float(ncc[u, v]), su, sv, edge


def consistency(cps: np.ndarray, priors=None) -> np.ndarray:
    """Median-translation consistency (the translation special case of the
    outlier rejection of Section 3.2.3) at the 1.5 px threshold of Section 4.1.
    Sets INCONSISTENT and VALID in place and returns cps."""
    n = len(cps)
    py = np.zeros(n) if priors is None else np.asarray(priors)[:, 0].astype(np.float64)
    px = np.zeros(n) if priors is None else np.asarray(priors)[:, 1].astype(np.float64)
    bad = OOB | FLAT_T | FLAT_S | EDGE_PEAK | NONFINITE
    elig = (cps["flags"] & bad) == 0
    if not elig.any():
        return cps
    ty = py + cps["dy"] + cps["sub_dy"]
    tx = px + cps["dx"] + cps["sub_dx"]
    my, mx = np.median(ty[elig]), np.median(tx[elig])
    dev = np.hypot(ty - my, tx - mx)
    for i in np.nonzero(elig)[0]:
        if dev[i] > CONSISTENCY_PX:
            cps["flags"][i] |= INCONSISTENT
        else:
            cps["flags"][i] |= VALID
    return cps


def decide(ncc: np.ndarray, flatT: bool, nonfinite: bool, r: int):
    """Per-CP decision from one NCC surface (Section 3.2.2: the most similar
    position is the CP): (dy, dx, sub_dy, sub_dx, score, flags), before the
    consistency check."""
    if nonfinite:
        return 0, 0, 0.0, 0.0, 0.0, NONFINITE
    if flatT:
        return 0, 0, 0.0, 0.0, 0.0, FLAT_T
    if not np.any(ncc != 0.0):
        return 0, 0, 0.0, 0.0, 0.0, FLAT_S
    u, v, sc, su, sv, edge = peak(ncc)
    return u - r, v - r, su, sv, sc, (EDGE_PEAK if edge else 0)


def match(Fs: np.ndarray, Fr: np.ndarray, ips, m: int, r: int, prior=None,
          method: str = "fast", integ=None, want_surfaces: bool = False):
    """CP detection by template matching (Section 3.2.2): template around each
    IP in the sensed descriptor, search window in the reference descriptor.

    Fs, Fr: (H, W, z) descriptors.  ips: (n, 2) (row, col).  prior: (n, 2) or
    None.  method: "fast" (Eq. 9-16) or "brute" (Eq. 8).  integ: optional
    (G1, G2) of Fr.  Returns the CP array (and the NCC surfaces)."""
    ips = np.asarray(ips)
    n = len(ips)
    Hs, Ws, _ = Fs.shape
    Hr, Wr, _ = Fr.shape
    M = m + 2 * r
    V = 2 * r + 1
    cps = np.zeros(n, dtype=CP_DTYPE)
    surfaces = np.zeros((n, V, V))
    if method == "fast" and integ is None:
        integ = integral_feature_images(Fr)
    for i in range(n):
        cps["sen_row"][i], cps["sen_col"][i] = ips[i]
        pr = None if prior is None else prior[i]
        (ty, tx), (sy, sx) = window_origins(ips[i], pr, m, r)
        if not (in_bounds(ty, tx, m, m, Hs, Ws) and in_bounds(sy, sx, M, M, Hr, Wr)):
            cps["flags"][i] = OOB
            continue
        T = Fs[ty:ty + m, tx:tx + m, :]
        S = Fr[sy:sy + M, sx:sx + M, :]
        if method == "brute":
            nonfin = not (np.all(np.isfinite(T)) and np.all(np.isfinite(S)))
            ncc, flatT = (np.zeros((V, V)), False) if nonfin else ncc_bruteforce(S, T)
        else:
            ncc, flatT, nonfin = ncc_fast(S, T, integ[0], integ[1], (sy, sx))
        surfaces[i] = ncc
        (cps["dy"][i], cps["dx"][i], cps["sub_dy"][i], cps["sub_dx"][i],
         cps["score"][i], cps["flags"][i]) = decide(ncc, flatT, nonfin, r)
    consistency(cps, prior)
    return (cps, surfaces) if want_surfaces else cps


def quantiser(kind):
    """None, "bf16" or "f16": the rounding of the stored descriptor (float64
    -> float32 -> storage type), as a function on arrays."""
    if kind is None:
        return lambda a: a
    q = round_to_bf16 if kind == "bf16" else round_to_f16
    return lambda a: q(np.asarray(a, np.float32)).astype(np.float64)


def match_one_region(ref: np.ndarray, sen: np.ndarray, ip, m: int, r: int, p: Params | None = None,
                     prior=None, quantise=None):
    """One CP of register_cps (before the consistency check) computed from
    crops only: SFOC of the template and search windows by sfoc_region
    (optionally rounded to the storage type), NCC by Eq. 9-16 with integral
    images built over the search window.  Returns (record, surface) with
    record = (dy, dx, sub_dy, sub_dx, score, flags)."""
    p = p or Params()
    (ty, tx), (sy, sx) = window_origins(ip, prior, m, r)
    M = m + 2 * r
    if not (in_bounds(ty, tx, m, m, *sen.shape) and in_bounds(sy, sx, M, M, *ref.shape)):
        return (0, 0, 0.0, 0.0, 0.0, OOB), np.zeros((2 * r + 1, 2 * r + 1))
    q = quantiser(quantise)
    T = q(sfoc_region(sen, ty, tx, m, m, p))
    S = q(sfoc_region(ref, sy, sx, M, M, p))
    ncc, flatT, nonfin = ncc_fast(S, T)
    return decide(ncc, flatT, nonfin, r), ncc


def match_one_region_variants(ref: np.ndarray, sen: np.ndarray, ip, m: int, r: int, p: Params | None = None,
                              prior=None, quantise=(None,)):
    """match_one_region for several storage roundings of the same CP: the
    template and search-window descriptors (Section 2.1) are computed once,
    then each rounding in `quantise` (None, "bf16", "f16") is applied to
    both and Eq. 9-16 plus the peak decision run on the rounded values.
    Returns a list of (record, surface), one per entry of `quantise`, each
    equal to what match_one_region returns for that rounding."""
    p = p or Params()
    (ty, tx), (sy, sx) = window_origins(ip, prior, m, r)
    M = m + 2 * r
    if not (in_bounds(ty, tx, m, m, *sen.shape) and in_bounds(sy, sx, M, M, *ref.shape)):
        return [((0, 0, 0.0, 0.0, 0.0, OOB), np.zeros((2 * r + 1, 2 * r + 1))) for _ in quantise]
    T0 = sfoc_region(sen, ty, tx, m, m, p)
    S0 = sfoc_region(ref, sy, sx, M, M, p)
    out = []
    for kind in quantise:
        q = quantiser(kind)
        ncc, flatT, nonfin = ncc_fast(q(S0), q(T0))
        out.append((decide(ncc, flatT, nonfin, r), ncc))
    return out


def register_cps(ref: np.ndarray, sen: np.ndarray, ips, m: int, r: int,
                 p: Params | None = None, prior=None, method: str = "fast",
                 quantise=None, want_surfaces: bool = False):
    """Fine registration of one pair: SFOC of both images, then matching.
    quantise: None, "bf16" or "f16" rounds the stored descriptor first."""
    p = p or Params()
    Fr = sfoc(ref, p)
    Fs = sfoc(sen, p)
    q = quantiser(quantise)
    return match(q(Fs), q(Fr), ips, m, r, prior, method, want_surfaces=want_surfaces)


# ------------------------------------------------------ cost model ---------
def cost_fast(M: int, N: int, z: int) -> float:
    """Eq. 17: T1 ~ 4 M N z log2(M N z) multiplications."""
    return 4.0 * M * N * z * math.log2(M * N * z)


def cost_direct(m: int, n: int, M: int, N: int, z: int) -> float:
    """Eq. 18: T2 = 3 m n z (M - m + 1)(N - n + 1)."""
    return 3.0 * m * n * z * (M - m + 1) * (N - n + 1)


def cost_ratio(m: int, M: int, z: int) -> float:
    """Eq. 19 with square windows."""
    return cost_fast(M, M, z) / cost_direct(m, m, M, M, z)
