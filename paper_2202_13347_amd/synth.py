"""Seeded synthetic multimodal image pairs and interest-point layouts.

This module only draws inputs: piecewise-constant scenes, intensity remaps,
noise and shifts.  It holds none of the matching method's arithmetic, so both
the GPU path and the CPU reference can be fed from it.

The paper's own image pairs (optical / infrared / LiDAR / SAR / map, Section
4.1, Table 1) are not available; these scenes stand in for them.  Each pair
is a reference image and a "sensed" image that sees the same scene through
a different, non-monotonic intensity response per region (nonlinear
radiometric difference), with contrast reversed in half of the regions,
additive noise, optional multiplicative gamma speckle (a SAR-like look
count) and a known translation with a sub-pixel fraction.  After a
correct match, the sensed point p corresponds to the reference point p + d.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import fft as sfft
from scipy import ndimage


@dataclass
class Pair:
    ref: np.ndarray        # (H, W) float32
    sen: np.ndarray        # (H, W) float32
    shift: np.ndarray      # (2,) float64, (dy, dx): sen(p) <-> ref(p + shift)
    seed: int


def _convex_polygon(rng, h, w, cy, cx, rad):
    """Random convex polygon (3..7 vertices) of radius ~rad: its clipped
    bounding box (y0, y1, x0, x1) and the inside mask over that box."""
    nv = int(rng.integers(3, 8))
    ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
    rr = rad * rng.uniform(0.6, 1.0, nv)
    vy = cy + rr * np.sin(ang)
    vx = cx + rr * np.cos(ang)
    y0 = int(max(0, np.floor(vy.min()))); y1 = int(min(h, np.ceil(vy.max()) + 1))
    x0 = int(max(0, np.floor(vx.min()))); x1 = int(min(w, np.ceil(vx.max()) + 1))
    if y1 <= y0 or x1 <= x0:
        return y0, y0, x0, x0, None
    yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    inside = np.ones(yy.shape, dtype=bool)
    for i in range(nv):
        j = (i + 1) % nv
        ex, ey = vx[j] - vx[i], vy[j] - vy[i]
        inside &= (ex * (yy - vy[i]) - ey * (xx - vx[i])) >= 0
    return y0, y1, x0, x1, inside


def _label_map(rng, h, w, n_shapes, size_lo, size_hi):
    """Painter's-algorithm region labels: 0 = background, k = k-th shape."""
    lab = np.zeros((h, w), dtype=np.int32)
    for k in range(1, n_shapes + 1):
        sz = rng.uniform(size_lo, size_hi)
        cy = rng.uniform(0, h); cx = rng.uniform(0, w)
        if rng.random() < 0.5:
            hh = sz * rng.uniform(0.4, 1.0); ww = sz * rng.uniform(0.4, 1.0)
            y0 = int(max(0, cy - hh / 2)); y1 = int(min(h, cy + hh / 2))
            x0 = int(max(0, cx - ww / 2)); x1 = int(min(w, cx + ww / 2))
            lab[y0:y1, x0:x1] = k
        else:
            y0, y1, x0, x1, inside = _convex_polygon(rng, h, w, cy, cx, sz / 2)
            if inside is not None:
                lab[y0:y1, x0:x1][inside] = k
    return lab


def _value_noise(rng, h, w, cell, std):
    """Smooth noise: a coarse random grid upsampled bilinearly."""
    gh = h // cell + 4; gw = w // cell + 4
    g = rng.standard_normal((gh, gw)).astype(np.float32)
    up = ndimage.zoom(g, cell, order=1)[:h, :w]
    s = up.std()
    return up * (std / s) if s > 0 else up


def _blur_shift(img, sigma, shift):
    """Gaussian blur (standard deviation sigma) and a translation by shift =
    (dy, dx), out(y, x) = blurred(y - dy, x - dx) on a periodic canvas, in one
    Fourier-domain product."""
    H, W = img.shape
    F = sfft.rfft2(img, workers=-1)
    ky = sfft.fftfreq(H)[:, None]
    kx = sfft.rfftfreq(W)[None, :]
    g = np.exp(-2.0 * (np.pi * sigma) ** 2 * (ky * ky + kx * kx))
    ph = np.exp(-2j * np.pi * (ky * shift[0] + kx * shift[1]))
    return sfft.irfft2(F * (g * ph), s=(H, W), workers=-1)


def _cubic_maps(rng, n):
    """Per-region random non-monotonic cubic intensity responses on [0, 1]."""
    coef = rng.uniform(-2.0, 2.0, size=(n, 4))
    v = np.linspace(0, 1, 65)
    out = []
    for c in coef:
        y = c[0] + c[1] * v + c[2] * v ** 2 + c[3] * v ** 3
        lo, hi = y.min(), y.max()
        if hi - lo < 1e-3:
            c = np.array([0.0, 1.0, 0.0, 0.0]); lo, hi = 0.0, 1.0
        out.append((c, lo, hi))
    return out


def _apply_maps(scene, lab, maps, flip, rows=512):
    """Per-region response: the region's cubic applied to the reference
    intensity, normalised by its range on [0, 1], reversed where flipped.
    Evaluated in row bands to bound memory."""
    coef = np.array([c for c, _, _ in maps])                      # (k, 4)
    lo = np.array([l for _, l, _ in maps])
    span = np.array([h - l for _, l, h in maps])
    out = np.empty_like(scene)
    for y0 in range(0, scene.shape[0], rows):
        v = scene[y0:y0 + rows]
        k = lab[y0:y0 + rows]
        c = coef[k]
        y = (c[..., 0] + v * (c[..., 1] + v * (c[..., 2] + v * c[..., 3])) - lo[k]) / span[k]
        out[y0:y0 + rows] = np.where(flip[k], 1.0 - y, y)
    return out


def make_pair(seed: int, size: int | tuple[int, int], max_shift: float,
              speckle_looks: int = 0, n_shapes: int | None = None,
              noise_std: float = 0.05, integer_shift: bool = False) -> Pair:
    """One seeded multimodal pair.

    The reference is a painter's-algorithm layout of rectangles and convex
    polygons with U[0, 1] intensities plus smooth value noise (standard
    deviation 0.1), blurred with a Gaussian of standard deviation 1.  The
    sensed image applies to the same (unblurred) reference intensities a
    per-region random non-monotonic cubic response, reversed in half of the
    regions, is blurred the same way and translated, then gets additive
    N(0, noise_std^2) noise and optional Gamma(L, 1/L) speckle.

    size          : side (or (H, W)) of both images.
    max_shift     : the true shift is drawn from U[-max_shift, max_shift]^2.
    speckle_looks : if > 0, the sensed image is multiplied by Gamma(L, 1/L).
    n_shapes      : regions; default 40 per 256x256 of area.
    integer_shift : round the drawn shift to whole pixels.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    H, W = (size, size) if np.isscalar(size) else size
    if n_shapes is None:
        n_shapes = max(8, int(round(40 * H * W / 256.0 ** 2)))
    shift = rng.uniform(-max_shift, max_shift, size=2)
    if integer_shift:
        shift = np.round(shift)
    pad = int(np.ceil(max_shift)) + 8
    ch, cw = H + 2 * pad, W + 2 * pad
    lab = _label_map(rng, ch, cw, n_shapes, 8.0, min(96.0, max(16.0, min(H, W) / 2)))
    vals = rng.uniform(0, 1, n_shapes + 1)
    maps = _cubic_maps(rng, n_shapes + 1)
    flip = rng.random(n_shapes + 1) < 0.5
    scene_r = vals[lab] + _value_noise(rng, ch, cw, 16, 0.1)
    scene_s = _apply_maps(scene_r, lab, maps, flip)
    # sen(y, x) = blurred scene_s(y + dy, x + dx): translate by -d.  The
    # canvas margin exceeds the shift, so the periodic wrap stays outside.
    scene_r = _blur_shift(scene_r, 1.0, (0.0, 0.0))
    if integer_shift:
        dy, dx = int(shift[0]), int(shift[1])
        sen_c = np.roll(_blur_shift(scene_s, 1.0, (0.0, 0.0)), (-dy, -dx), axis=(0, 1))
    else:
        sen_c = _blur_shift(scene_s, 1.0, (-shift[0], -shift[1]))
    ref = scene_r[pad:pad + H, pad:pad + W]
    sen = sen_c[pad:pad + H, pad:pad + W]
    if noise_std > 0:
        sen = sen + rng.normal(0.0, noise_std, sen.shape)
    if speckle_looks > 0:
        L = float(speckle_looks)
        sen = sen * rng.gamma(L, 1.0 / L, sen.shape)
    return Pair(ref=np.ascontiguousarray(ref, dtype=np.float32),
                sen=np.ascontiguousarray(sen, dtype=np.float32),
                shift=shift.astype(np.float64), seed=seed)


def grid_ips(H: int, W: int, n_side: int, margin: int) -> np.ndarray:
    """n_side x n_side interest points evenly spaced in [margin, side-1-margin],
    as an (n, 2) int32 array of (row, col)."""
    ys = np.round(np.linspace(margin, H - 1 - margin, n_side)).astype(np.int32)
    xs = np.round(np.linspace(margin, W - 1 - margin, n_side)).astype(np.int32)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], axis=1).astype(np.int32)


def random_ips(seed: int, H: int, W: int, n: int, margin: int) -> np.ndarray:
    """n seeded uniform interest points inside the margin, (n, 2) int32."""
    rng = np.random.default_rng(np.random.PCG64(seed + 7919))
    ys = rng.integers(margin, H - margin, n)
    xs = rng.integers(margin, W - margin, n)
    return np.stack([ys, xs], axis=1).astype(np.int32)


# Workload recipes (image side, IP grid, template m, search radius r, shift bound).
SMALL = dict(size=256, n_side=4, m=32, r=10, max_shift=8.0, speckle=0)
SCENE = dict(size=2048, n_side=20, m=64, r=32, max_shift=30.0, speckle=4)
LARGE = dict(size=10000, n_side=71, m=64, r=48, max_shift=44.0, speckle=4, n_ips=5000)


# Batching workload: 64 pairs of uneven square sides U{512..4096}, 50..500
# seeded uniform IPs each, template sides from {48, 64, 96} and radii from
# {16, 32, 64} per pair, shift bound r - 2, every second pair speckled.
BATCH = dict(n_pairs=64, side=(512, 4096), n_ips=(50, 500), m=(48, 64, 96), r=(16, 32, 64), speckle=4)


def _pool(workers: int):
    """Process pool of forked workers (NumPy only; they never exec, so a
    parent that already uses the GPU can fan out input generation)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    return ProcessPoolExecutor(max_workers=max(1, workers), mp_context=multiprocessing.get_context("fork"))


def batch_specs(seed: int, recipe: dict = BATCH) -> list[dict]:
    """Per-pair draws of the batching workload (no images): seed, side, m,
    r, shift bound, speckle looks and IP count."""
    rng = np.random.default_rng(np.random.PCG64(seed + 424242))
    out = []
    for k in range(recipe["n_pairs"]):
        side = int(rng.integers(recipe["side"][0], recipe["side"][1] + 1))
        m = int(rng.choice(recipe["m"]))
        r = int(rng.choice(recipe["r"]))
        n = int(rng.integers(recipe["n_ips"][0], recipe["n_ips"][1] + 1))
        out.append(dict(seed=seed * 1000 + k, side=side, m=m, r=r, max_shift=float(r - 2),
                        speckle=recipe["speckle"] if k % 2 else 0, n=n))
    return out


def batch_pair(spec: dict):
    """(pair, ips) of one batching spec; IPs uniform within the margin."""
    p = make_pair(spec["seed"], spec["side"], spec["max_shift"], speckle_looks=spec["speckle"])
    b = (spec["m"] + 1) // 2 + spec["r"]
    ips = random_ips(spec["seed"], spec["side"], spec["side"], spec["n"], b)
    return p, ips


def batch_workload(seed: int, recipe: dict = BATCH, workers: int = 8):
    """[(spec, pair, ips)] for the batching workload, generated in a
    process pool."""
    specs = batch_specs(seed, recipe)
    order = sorted(range(len(specs)), key=lambda k: -specs[k]["side"])   # big ones first
    with _pool(workers) as ex:
        res = dict(zip(order, ex.map(batch_pair, [specs[k] for k in order])))
    return [(specs[k], res[k][0], res[k][1]) for k in range(len(specs))]


# Learned-head training pairs: 512 x 512, ~100 uniform IPs, m 64, r 32,
# 30% of the pairs with occlusion patches pasted on the sensed image.
HEAD = dict(size=512, n_ips=100, m=64, r=32, occluded=0.3, speckle=4)


def occlude(sen: np.ndarray, seed: int, n_patches=(2, 5), side=(48, 128)):
    """Paste 2..4 rectangles of unrelated texture (smooth noise at a random
    level) onto a copy of the sensed image.  Returns (image, mask of the
    pasted pixels)."""
    rng = np.random.default_rng(np.random.PCG64(seed + 99991))
    H, W = sen.shape
    out = sen.copy()
    mask = np.zeros((H, W), dtype=bool)
    for _ in range(int(rng.integers(*n_patches))):
        h = int(rng.integers(side[0], side[1] + 1))
        w = int(rng.integers(side[0], side[1] + 1))
        y0 = int(rng.integers(0, max(1, H - h)))
        x0 = int(rng.integers(0, max(1, W - w)))
        tex = _value_noise(rng, h, w, 8, 0.3) + rng.uniform(0.0, 1.0)
        out[y0:y0 + h, x0:x0 + w] = tex
        mask[y0:y0 + h, x0:x0 + w] = True
    return out.astype(np.float32), mask


def head_pair(seed: int, recipe: dict = HEAD):
    """(pair, ips, occlusion mask or None) of one head-training seed."""
    rng = np.random.default_rng(np.random.PCG64(seed + 31337))
    occluded = rng.random() < recipe["occluded"]
    p = make_pair(seed, recipe["size"], float(recipe["r"] - 2),
                  speckle_looks=recipe["speckle"] if rng.random() < 0.5 else 0)
    b = (recipe["m"] + 1) // 2 + recipe["r"]
    ips = random_ips(seed, recipe["size"], recipe["size"], recipe["n_ips"], b)
    mask = None
    if occluded:
        sen, mask = occlude(p.sen, seed)
        p = Pair(ref=p.ref, sen=sen, shift=p.shift, seed=p.seed)
    return p, ips, mask


def head_pairs(seeds, recipe: dict = HEAD, workers: int = 8):
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 4:
        return [head_pair(s, recipe) for s in seeds]
    with _pool(workers) as ex:
        return list(ex.map(head_pair, seeds, [recipe] * len(seeds), chunksize=8))


def head_init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters of the learned head (float32, the order of
    the header): He-uniform weights with bound sqrt(6 / fan_in), zero
    biases."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    parts = []
    for shape in [(32, 1, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,),
                  (32, 808), (32,), (3, 32), (3,)]:
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.uniform(-1.0, 1.0, shape) * np.sqrt(6.0 / fan_in))
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)


def ransac_words(seed: int, n_hyp: int, k: int) -> np.ndarray:
    """n_hyp * k uniform 32-bit random words (the sample draws of RANSAC)."""
    rng = np.random.default_rng(np.random.PCG64(seed + 7919))
    return rng.integers(0, 2 ** 32, n_hyp * k, dtype=np.uint64).astype(np.uint32)


# Pairs related by a projective map: a rotation about the image centre, a
# scale, a translation and a small perspective term, with occlusion patches
# on the sensed image (the mismatches that outlier rejection removes).
WARP = dict(size=2048, n_side=20, m=64, r=32, rot_deg=0.75, scale=0.004, persp=1e-6, max_shift=5.0, speckle=4,
            occluded=True)


@dataclass
class WarpPair:
    ref: np.ndarray        # (H, W) float32
    sen: np.ndarray        # (H, W) float32
    model: np.ndarray      # (3, 3) float64: sensed (row, col, 1) -> reference, entry (2, 2) = 1
    mask: np.ndarray | None   # occluded sensed pixels
    seed: int


def warp_model(rng, size: int, rot_deg: float, scale: float, persp: float, max_shift: float) -> np.ndarray:
    """Random projective map in (row, col) pixels about the image centre;
    the rotation and scale change have magnitudes in [1/2, 1] of their
    bounds, with random signs."""
    a = np.deg2rad(rot_deg * rng.uniform(0.5, 1.0) * rng.choice([-1.0, 1.0]))
    sc = 1.0 + scale * rng.uniform(0.5, 1.0) * rng.choice([-1.0, 1.0])
    t = rng.uniform(-max_shift, max_shift, 2)
    g, h = rng.uniform(-persp, persp, 2)
    c = 0.5 * (size - 1)
    R = np.array([[sc * np.cos(a), -sc * np.sin(a), 0.0], [sc * np.sin(a), sc * np.cos(a), 0.0], [0.0, 0.0, 1.0]])
    K = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [g, h, 1.0]])
    C = np.array([[1.0, 0.0, c], [0.0, 1.0, c], [0.0, 0.0, 1.0]])
    Ci = np.array([[1.0, 0.0, -c], [0.0, 1.0, -c], [0.0, 0.0, 1.0]])
    T = np.array([[1.0, 0.0, t[0]], [0.0, 1.0, t[1]], [0.0, 0.0, 1.0]])
    M = T @ C @ K @ R @ Ci
    return M / M[2, 2]


def apply_model(M: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """(n, 2) (row, col) points through a 3x3 projective map."""
    q = np.column_stack([pts, np.ones(len(pts))]) @ np.asarray(M).T
    return q[:, :2] / q[:, 2:3]


def make_warp_pair(seed: int, recipe: dict = WARP, noise_std: float = 0.05) -> WarpPair:
    """A multimodal pair as make_pair draws it (regions, per-region cubic
    responses, blur, noise, speckle) whose sensed pixel p shows the scene
    point that the reference shows at model(p): the blurred sensed scene is
    resampled (cubic spline) at model(p)."""
    rng = np.random.default_rng(np.random.PCG64(seed + 424243))
    size = recipe["size"]
    M = warp_model(rng, size, recipe["rot_deg"], recipe["scale"], recipe["persp"], recipe["max_shift"])
    corners = np.array([[0, 0], [0, size - 1], [size - 1, 0], [size - 1, size - 1]], np.float64)
    reach = np.abs(apply_model(M, corners) - corners).max()
    pad = int(np.ceil(reach)) + 16
    ch = cw = size + 2 * pad
    n_shapes = max(8, int(round(40 * size * size / 256.0 ** 2)))
    lab = _label_map(rng, ch, cw, n_shapes, 8.0, min(96.0, max(16.0, size / 2)))
    vals = rng.uniform(0, 1, n_shapes + 1)
    maps = _cubic_maps(rng, n_shapes + 1)
    flip = rng.random(n_shapes + 1) < 0.5
    scene_r = vals[lab] + _value_noise(rng, ch, cw, 16, 0.1)
    scene_s = _blur_shift(_apply_maps(scene_r, lab, maps, flip), 1.0, (0.0, 0.0))
    scene_r = _blur_shift(scene_r, 1.0, (0.0, 0.0))
    ref = scene_r[pad:pad + size, pad:pad + size]
    sen = np.empty((size, size), np.float64)
    cols = np.arange(size, dtype=np.float64)
    for y0 in range(0, size, 256):
        rows = np.arange(y0, min(size, y0 + 256), dtype=np.float64)
        pts = np.stack(np.meshgrid(rows, cols, indexing="ij"), -1).reshape(-1, 2)
        q = apply_model(M, pts) + pad
        sen[y0:y0 + len(rows)] = ndimage.map_coordinates(scene_s, q.T, order=3, mode="nearest").reshape(len(rows), size)
    if noise_std > 0:
        sen = sen + rng.normal(0.0, noise_std, sen.shape)
    if recipe.get("speckle", 0) > 0:
        L = float(recipe["speckle"])
        sen = sen * rng.gamma(L, 1.0 / L, sen.shape)
    mask = None
    if recipe.get("occluded"):
        sen, mask = occlude(sen.astype(np.float32), seed, n_patches=(4, 9), side=(96, 256))
    return WarpPair(ref=np.ascontiguousarray(ref, np.float32), sen=np.ascontiguousarray(sen, np.float32), model=M,
                    mask=mask, seed=seed)


# Noise sensitivity: the levels of the paper's sweep (Gaussian white noise of
# variance 0..0.01 in steps of 0.001, speckle of variance 0..0.1 in steps of
# 0.01) on seeded pairs matched with 80 x 80 templates.
SWEEP = dict(size=768, n_pairs=8, m=80, r=20, blocks=(10, 20), fast_threshold=0.05,
             gaussian=[round(0.001 * i, 3) for i in range(11)], speckle=[round(0.01 * i, 2) for i in range(11)])


def gaussian_noise(img: np.ndarray, v: float, seed: int) -> np.ndarray:
    """img + N(0, v) (v is the variance), float32."""
    rng = np.random.default_rng(np.random.PCG64(seed + 5003))
    return (img + rng.normal(0.0, np.sqrt(v), img.shape)).astype(np.float32)


def speckle_noise(img: np.ndarray, v: float, seed: int) -> np.ndarray:
    """img * (1 + n), n uniform with mean 0 and variance v, float32."""
    rng = np.random.default_rng(np.random.PCG64(seed + 7001))
    h = np.sqrt(3.0 * v)
    return (img * (1.0 + rng.uniform(-h, h, img.shape))).astype(np.float32)


def sweep_pair(seed: int, recipe: dict = SWEEP) -> Pair:
    return make_pair(seed, recipe["size"], float(recipe["r"] - 4))


def workload(recipe: dict, seed: int):
    """(pair, ips, m, r) for a recipe; IP margin = ceil(m/2) + r."""
    p = make_pair(seed, recipe["size"], recipe["max_shift"], speckle_looks=recipe["speckle"])
    b = (recipe["m"] + 1) // 2 + recipe["r"]
    ips = grid_ips(recipe["size"], recipe["size"], recipe["n_side"], b)
    if "n_ips" in recipe:
        ips = ips[:recipe["n_ips"]]
    return p, ips, recipe["m"], recipe["r"]
