"""Host-side logic of batched plans (no GPU): struct layouts, transform-side
candidates, the sensed tiles and argument rejection in
sfoc_plan_create."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2202_13347_amd import sfoc as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x1000   # never dereferenced: every call below fails validation first


def test_pair_and_info_layout_match_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "sfoc.h"
#define P(f) printf("pair.%s %zu\n", #f, offsetof(sfoc_pair, f));
#define I(f) printf("info.%s %zu\n", #f, offsetof(sfoc_plan_info, f));
int main(void) {
  P(ref) P(Hr) P(Wr) P(ldr) P(sen) P(Hs) P(Ws) P(lds) P(ips) P(prior) P(n) P(m) P(r) P(fft_side) P(ncc) P(cps)
  I(n_pairs) I(describe_tiles) I(match_items) I(peak_items) I(tuned_classes) I(cached_classes) I(graph)
  I(persistent) I(describe_config) I(direct_items)
  I(device_bytes)
  printf("pair.size %zu\ninfo.size %zu\n", sizeof(sfoc_pair), sizeof(sfoc_plan_info));
  return 0;
}''')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for name, _ in S.Pair._fields_:
        assert int(got["pair." + name]) == getattr(S.Pair, name).offset, name
    for name, _ in S.PlanInfo._fields_:
        assert int(got["info." + name]) == getattr(S.PlanInfo, name).offset, name
    assert int(got["pair.size"]) == ctypes.sizeof(S.Pair)
    assert int(got["info.size"]) == ctypes.sizeof(S.PlanInfo)


SIDES = (64, 128, 160, 192)


def _split(m, r, L):
    """Offset blocks per axis for transform side L, written from the
    condition that a block of Vb offsets needs a search window of
    m + Vb - 1 <= L rows (None if no block of >= 2 offsets fits)."""
    V = 2 * r + 1
    best = None
    for Vb in range(V, 1, -1):
        if m + Vb - 1 <= L:
            best = Vb
            break
    if best is None:
        return None
    return math.ceil(V / best)


def _default(m, r):
    """The smallest side holding the whole window; beyond 192 the side of
    least transform work nb^2 L^2 log2(L^2)."""
    M = m + 2 * r
    for L in SIDES:
        if M <= L:
            return L
    cost = {L: _split(m, r, L) ** 2 * L * L * math.log2(L * L) for L in SIDES if _split(m, r, L)}
    return min(cost, key=cost.get) if cost else None


@pytest.mark.parametrize("m,r", [(32, 10), (48, 16), (64, 32), (96, 64), (48, 64), (30, 100), (64, 16),
                                 (96, 16), (3, 1), (126, 200), (60, 2), (62, 40), (64, 48), (150, 20),
                                 (191, 1), (100, 46), (16, 100), (190, 300)])
def test_match_candidates(m, r):
    got = S.match_candidates(m, r)
    d = _default(m, r)
    assert got[0] == (d, _split(m, r, d))
    want = [(L, _split(m, r, L)) for L in SIDES if L != d and _split(m, r, L) is not None and _split(m, r, L) <= 8]
    assert got[1:] == want, (got, want)


def test_large_windows_are_one_transform():
    # every search window up to 192 x 192 is a single transform
    for m, r in ((64, 48), (32, 60), (100, 46), (150, 20), (126, 2)):
        L, nb = S.match_candidates(m, r)[0]
        assert nb == 1 and L >= m + 2 * r and L in (160, 192)
    # 224: 2 x 2 blocks of the 160 side (4 x 160^2 transforms, less work than 4 x 192^2 or 16 x 128^2)
    assert S.match_candidates(96, 64)[0] == (160, 2)


def test_match_candidates_unsupported():
    assert S.match_candidates(2, 4) == []      # m < 3
    assert S.match_candidates(192, 10) == []   # m > 191
    assert S.match_candidates(30, 512) == []   # r > 511


def _in_bounds(ips, prior, m, r, Hs, Ws, Hr, Wr):
    """Top-left corners of the templates of the IPs whose template and
    search window stay inside their images."""
    M = m + 2 * r
    out = []
    for i, (y, x) in enumerate(ips):
        ty, tx = int(y) - m // 2, int(x) - m // 2
        py, px = (prior[i] if prior is not None else (0, 0))
        sy, sx = ty - r + int(py), tx - r + int(px)
        if ty < 0 or tx < 0 or ty + m > Hs or tx + m > Ws:
            continue
        if sy < 0 or sx < 0 or sy + M > Hr or sx + M > Wr:
            continue
        out.append((ty, tx))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_sensed_tiles_cover_the_templates(seed):
    rng = np.random.default_rng(seed)
    Hs, Ws = int(rng.integers(100, 300)), int(rng.integers(100, 300))
    Hr, Wr = int(rng.integers(100, 300)), int(rng.integers(100, 300))
    m, r = int(rng.integers(3, 80)), int(rng.integers(1, 20))
    n = 40
    ips = np.stack([rng.integers(-10, Hs + 10, n), rng.integers(-10, Ws + 10, n)], 1).astype(np.int32)
    prior = rng.integers(-15, 16, (n, 2)).astype(np.int32) if seed else None
    got = S.sensed_tiles(ips, m, r, Hs, Ws, Hr, Wr, prior)
    tl = [tuple(map(int, t)) for t in got]
    assert len(set(tl)) == len(tl)                                     # distinct
    for (y, x) in tl:                                                   # inside the image
        assert 0 <= y < Hs and 0 <= x < Ws
    # every template pixel of an in-bounds IP is described by some tile ...
    cov = np.zeros((Hs, Ws), dtype=bool)
    for (y, x) in tl:
        cov[y:y + 32, x:x + 32] = True
    need = np.zeros((Hs, Ws), dtype=bool)
    tops = _in_bounds(ips, prior, m, r, Hs, Ws, Hr, Wr)
    for (ty, tx) in tops:
        need[ty:ty + m, tx:tx + m] = True
    assert not (need & ~cov).any()
    # ... and every tile is one of some template's tiles: rows and columns
    # from its top-left corner in steps of 32
    for (y, x) in tl:
        assert any((y - ty) % 32 == 0 and 0 <= y - ty < m and (x - tx) % 32 == 0 and 0 <= x - tx < m
                   for (ty, tx) in tops), (y, x)
    # at most ceil(m/32)^2 tiles per in-bounds IP
    k = -(-m // 32)
    assert len(tl) <= len(tops) * k * k
    if not tops:
        assert len(tl) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sensed_grid_tiles_match_brute_force(seed):
    rng = np.random.default_rng(seed + 10)
    Hs, Ws = int(rng.integers(100, 300)), int(rng.integers(100, 300))
    Hr, Wr = int(rng.integers(100, 300)), int(rng.integers(100, 300))
    m, r = int(rng.integers(3, 80)), int(rng.integers(1, 20))
    n = 60
    ips = np.stack([rng.integers(-10, Hs + 10, n), rng.integers(-10, Ws + 10, n)], 1).astype(np.int32)
    prior = rng.integers(-15, 16, (n, 2)).astype(np.int32) if seed else None
    # the grid cover: every 32-grid tile holding a template pixel, row-major
    mask = np.zeros(((Hs + 31) // 32, (Ws + 31) // 32), dtype=bool)
    for (ty, tx) in _in_bounds(ips, prior, m, r, Hs, Ws, Hr, Wr):
        for yy in range(ty, ty + m):
            for xx in range(tx, tx + m):
                mask[yy // 32, xx // 32] = True
    want = np.argwhere(mask) * 32
    grid = S.sensed_tiles(ips, m, r, Hs, Ws, Hr, Wr, prior, S.COVER_GRID)
    np.testing.assert_array_equal(grid, want)
    tmpl = S.sensed_tiles(ips, m, r, Hs, Ws, Hr, Wr, prior, S.COVER_TEMPLATE)
    small = S.sensed_tiles(ips, m, r, Hs, Ws, Hr, Wr, prior, S.COVER_SMALLER)
    np.testing.assert_array_equal(small, grid if len(grid) < len(tmpl) else tmpl)


def test_sensed_tiles_cover_choice():
    # sparse IPs: each template's own tiles are fewer than the grid tiles it
    # touches; dense IPs: neighbours share grid tiles
    sparse = np.array([[100, 100], [300, 300]], np.int32)
    assert len(S.sensed_tiles(sparse, 64, 8, 512, 512, 512, 512)) == 2 * 2 * 2
    assert len(S.sensed_tiles(sparse, 64, 8, 512, 512, 512, 512, cover=S.COVER_GRID)) == 2 * 3 * 3
    dense = np.array([[y, x] for y in range(100, 200, 4) for x in range(100, 200, 4)], np.int32)
    g = S.sensed_tiles(dense, 64, 8, 512, 512, 512, 512, cover=S.COVER_GRID)
    t = S.sensed_tiles(dense, 64, 8, 512, 512, 512, 512)
    assert len(g) < len(t)
    np.testing.assert_array_equal(S.sensed_tiles(dense, 64, 8, 512, 512, 512, 512, cover=S.COVER_SMALLER), g)


def test_sensed_tiles_empty_and_errors():
    assert S.sensed_tiles(np.zeros((0, 2), np.int32), 16, 4, 64, 64, 64, 64).shape == (0, 2)
    with pytest.raises(S.SfocError):
        S.sensed_tiles(np.zeros((1, 2), np.int32), 2, 4, 64, 64, 64, 64)
    with pytest.raises(S.SfocError):
        S.sensed_tiles(np.zeros((1, 2), np.int32), 16, 4, 64, 64, 64, 64, cover=3)


def _pair(**kw):
    q = S.Pair()
    q.ref, q.Hr, q.Wr, q.ldr = FAKE, 64, 64, 64
    q.sen, q.Hs, q.Ws, q.lds = FAKE, 64, 64, 64
    q.ips, q.prior, q.n, q.m, q.r, q.fft_side = FAKE, None, 4, 16, 4, 0
    q.ncc, q.cps = None, FAKE
    for k, v in kw.items():
        setattr(q, k, v)
    return q


@pytest.mark.parametrize("kw,flags,code", [
    ({}, 32, S.SFOC_E_INVALID_ARG),                                # unknown flag
    ({"ref": None}, 0, S.SFOC_E_INVALID_ARG),
    ({"ldr": 10}, 0, S.SFOC_E_INVALID_ARG),
    ({"m": 2}, 0, S.SFOC_E_INVALID_ARG),
    ({"fft_side": 96}, 0, S.SFOC_E_INVALID_ARG),
    ({"m": 70, "r": 4, "fft_side": 64}, 0, S.SFOC_E_UNSUPPORTED),   # template wider than the transform
    ({"m": 192, "r": 10}, 0, S.SFOC_E_UNSUPPORTED),
    ({"cps": None}, 0, S.SFOC_E_INVALID_ARG),
    ({"Hs": 1 << 17}, 0, S.SFOC_E_UNSUPPORTED),
    ({"fft_side": S.MATCH_DIRECT}, 0, S.SFOC_E_UNSUPPORTED),        # the direct form needs 16-bit storage
    ({"fft_side": 2}, 0, S.SFOC_E_INVALID_ARG),
])
def test_plan_create_rejects_bad_pairs(kw, flags, code):
    arr = (S.Pair * 2)(_pair(), _pair(**kw))
    p = S.preset("baseline")
    h = ctypes.c_void_p(0)
    rc = S.lib().sfoc_plan_create(arr, 2, ctypes.byref(p), flags, None, None, ctypes.byref(h))
    assert rc == code
    assert not h.value


@pytest.mark.parametrize("kw", [{"r": 16}, {"m": 65, "r": 4}])
def test_plan_create_direct_form_limits(kw):
    # the direct form takes 2r + 1 <= 32 offsets per axis and m <= 64
    arr = (S.Pair * 1)(_pair(fft_side=S.MATCH_DIRECT, **kw))
    p = S.preset("baseline", dtype=S.DTYPE_BF16)
    h = ctypes.c_void_p(0)
    rc = S.lib().sfoc_plan_create(arr, 1, ctypes.byref(p), 0, None, None, ctypes.byref(h))
    assert rc == S.SFOC_E_UNSUPPORTED
    assert not h.value


def test_plan_create_rejects_empty_and_null():
    p = S.preset("baseline")
    h = ctypes.c_void_p(0)
    arr = (S.Pair * 1)(_pair())
    assert S.lib().sfoc_plan_create(arr, 0, ctypes.byref(p), 0, None, None, ctypes.byref(h)) == S.SFOC_E_INVALID_ARG
    assert S.lib().sfoc_plan_create(None, 1, ctypes.byref(p), 0, None, None, ctypes.byref(h)) == S.SFOC_E_INVALID_ARG
    assert S.lib().sfoc_plan_create(arr, 1, ctypes.byref(p), 0, None, None, None) == S.SFOC_E_INVALID_ARG
    bad = S.preset("baseline")
    bad.n_orient = 0
    assert S.lib().sfoc_plan_create(arr, 1, ctypes.byref(bad), 0, None, None, ctypes.byref(h)) == \
        S.SFOC_E_INVALID_ARG
    assert S.lib().sfoc_register_cps_batched(None, None) == S.SFOC_E_INVALID_ARG
    assert S.lib().sfoc_plan_destroy(None) == S.SFOC_E_INVALID_ARG


def test_streamed_workspace_query():
    p = S.preset("baseline")
    b = ctypes.c_size_t(0)
    q = S.lib().sfoc_register_streamed_workspace
    assert q(10000, 10000, 10000, 10000, 5000, 64, 48, 0, 0, ctypes.byref(p), ctypes.byref(b)) == S.SFOC_E_INVALID_ARG
    assert q(10000, 10000, 10000, 10000, 5000, 64, 48, 512, -1, ctypes.byref(p), ctypes.byref(b)) == \
        S.SFOC_E_INVALID_ARG
    assert q(10000, 10000, 10000, 10000, 5000, 2, 48, 512, 0, ctypes.byref(p), ctypes.byref(b)) == \
        S.SFOC_E_INVALID_ARG
    assert q(10000, 10000, 10000, 10000, 5000, 64, 48, 1024, 8, ctypes.byref(p), ctypes.byref(b)) == S.SFOC_OK
    band = b.value
    whole = S.register_workspace(10000, 10000, 10000, 10000, 5000, 64, 48, p)
    assert band < whole / 4
    # a band taller than the images needs what the whole-image call needs, plus the IP copies
    assert q(10000, 10000, 10000, 10000, 5000, 64, 48, 1 << 20, 8, ctypes.byref(p), ctypes.byref(b)) == S.SFOC_OK
    assert whole <= b.value <= whole + 2 * 5000 * 8 + 512
    assert S.lib().sfoc_register_cps_streamed(None, 10, 10, 10, None, 10, 10, 10, None, None, 0, 16, 4, 8, 0,
                                              ctypes.byref(p), None, None, None, 0, None) == S.SFOC_E_INVALID_ARG
