"""Host-side checks (no GPU) of the registration-system entry points around
the matching: RANSAC (parameter struct layout against the header, the
workspace query, argument rejection), rectification and block-based FAST
(argument rejection before anything is enqueued)."""
import ctypes
import os
import subprocess

import pytest

from paper_2202_13347_amd import sfoc as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def test_params_layout_matches_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "sfoc.h"
#define O(f) printf("%s %zu\n", #f, offsetof(sfoc_ransac_params, f));
int main(void) {
  O(model) O(n_hyp) O(n_refine) O(reserved) O(threshold) O(Hs) O(Ws) O(Hr) O(Wr)
  printf("size %zu\naffine %d\nprojective %d\nk %d\n", sizeof(sfoc_ransac_params), SFOC_MODEL_AFFINE,
         SFOC_MODEL_PROJECTIVE, SFOC_K_RANSAC);
  return 0;
}''')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for name, _ in S.RansacParams._fields_:
        assert int(got[name]) == getattr(S.RansacParams, name).offset, name
    assert int(got["size"]) == ctypes.sizeof(S.RansacParams)
    assert int(got["affine"]) == S.MODEL_AFFINE and int(got["projective"]) == S.MODEL_PROJECTIVE
    assert S.KERNEL_NAMES[int(got["k"])] == "ransac"


def _rp(**kw):
    rp = S.ransac_params(S.MODEL_PROJECTIVE, 100, (512, 512, 512, 512))
    for k, v in kw.items():
        setattr(rp, k, v)
    return rp


def test_workspace_grows_with_sizes():
    a = S.ransac_workspace(100, _rp())
    b = S.ransac_workspace(10000, _rp())
    c = S.ransac_workspace(100, _rp(n_hyp=100000))
    assert 0 < a < b and a < c
    assert S.ransac_workspace(0, _rp()) > 0


@pytest.mark.parametrize("kw,n,code", [
    ({"model": 7}, 10, S.SFOC_E_INVALID_ARG),
    ({"n_hyp": 0}, 10, S.SFOC_E_INVALID_ARG),
    ({"n_refine": -1}, 10, S.SFOC_E_INVALID_ARG),
    ({"n_refine": 17}, 10, S.SFOC_E_INVALID_ARG),
    ({"threshold": 0.0}, 10, S.SFOC_E_INVALID_ARG),
    ({"threshold": float("nan")}, 10, S.SFOC_E_INVALID_ARG),
    ({"Hr": 0}, 10, S.SFOC_E_INVALID_ARG),
    ({}, -1, S.SFOC_E_INVALID_ARG),
    ({}, (1 << 22) + 1, S.SFOC_E_UNSUPPORTED),
    ({"n_hyp": (1 << 20) + 1}, 10, S.SFOC_E_UNSUPPORTED),
])
def test_rejects_bad_arguments(kw, n, code):
    rp = _rp(**kw)
    b = ctypes.c_size_t(0)
    assert S.lib().sfoc_ransac_workspace(n, ctypes.byref(rp), ctypes.byref(b)) == code
    assert S.lib().sfoc_ransac_cps(FAKE, None, n, FAKE, ctypes.byref(rp), FAKE, 1 << 40, FAKE, FAKE, None, None,
                                   None) == code


def test_rejects_null_pointers_and_small_workspace():
    rp = _rp()
    L = S.lib()
    big = 1 << 40
    assert L.sfoc_ransac_workspace(10, None, None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_workspace(10, ctypes.byref(rp), None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(None, None, 10, FAKE, ctypes.byref(rp), FAKE, big, FAKE, FAKE, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(FAKE, None, 10, None, ctypes.byref(rp), FAKE, big, FAKE, FAKE, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(FAKE, None, 10, FAKE, None, FAKE, big, FAKE, FAKE, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(FAKE, None, 10, FAKE, ctypes.byref(rp), None, big, FAKE, FAKE, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(FAKE, None, 10, FAKE, ctypes.byref(rp), FAKE, big, None, FAKE, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    assert L.sfoc_ransac_cps(FAKE, None, 10, FAKE, ctypes.byref(rp), FAKE, big, FAKE, None, None, None,
                             None) == S.SFOC_E_INVALID_ARG
    need = S.ransac_workspace(10, rp)
    assert L.sfoc_ransac_cps(FAKE, None, 10, FAKE, ctypes.byref(rp), FAKE, need - 1, FAKE, FAKE, None, None,
                             None) == S.SFOC_E_WORKSPACE


def test_rectify_rejects_bad_arguments():
    L = S.lib()
    ok = dict(sen=FAKE, Hs=10, Ws=10, lds=10, model=FAKE, out=FAKE, Ho=10, Wo=10, ldo=10)

    def call(**kw):
        a = dict(ok, **kw)
        return L.sfoc_rectify(a["sen"], a["Hs"], a["Ws"], a["lds"], a["model"], a["out"], a["Ho"], a["Wo"], a["ldo"],
                              0.0, None)
    for kw in ({"sen": None}, {"model": None}, {"out": None}, {"Hs": 0}, {"Ws": 0}, {"lds": 9}, {"Ho": 0},
               {"Wo": 0}, {"ldo": 9}):
        assert call(**kw) == S.SFOC_E_INVALID_ARG, kw
    for kw in ({"Hs": (1 << 20) + 1}, {"Wo": (1 << 20) + 1, "ldo": (1 << 20) + 1},
               {"Hs": 1 << 16, "Ws": 1 << 15, "lds": 1 << 15}):
        assert call(**kw) == S.SFOC_E_UNSUPPORTED, kw
    assert S.KERNEL_NAMES[10] == "rectify"


def test_fast_rejects_bad_arguments():
    L = S.lib()
    b = ctypes.c_size_t(0)
    assert L.sfoc_fast_workspace(100, 100, 4, 4, 2, ctypes.byref(b)) == S.SFOC_OK and b.value >= 100 * 100 * 4
    assert L.sfoc_fast_workspace(100, 100, 4, 4, 2, None) == S.SFOC_E_INVALID_ARG
    ok = dict(img=FAKE, H=100, W=100, ld=100, thr=0.05, margin=10, nby=4, nbx=4, per=2, ips=FAKE, n_out=FAKE,
              ws=FAKE, wsb=1 << 40)

    def call(**kw):
        a = dict(ok, **kw)
        return L.sfoc_detect_ips(a["img"], a["H"], a["W"], a["ld"], a["thr"], a["margin"], a["nby"], a["nbx"],
                                 a["per"], a["ips"], None, None, a["n_out"], a["ws"], a["wsb"], None)
    for kw in ({"img": None}, {"ips": None}, {"n_out": None}, {"ws": None}, {"H": 0}, {"W": 0}, {"ld": 99},
               {"margin": -1}, {"thr": -0.1}, {"thr": float("inf")}, {"nby": 0}, {"nbx": 0}, {"per": 0}):
        assert call(**kw) == S.SFOC_E_INVALID_ARG, kw
    for kw in ({"per": 33}, {"nby": 257, "nbx": 256}, {"H": (1 << 20) + 1}):
        assert call(**kw) == S.SFOC_E_UNSUPPORTED, kw
    L.sfoc_fast_workspace(100, 100, 4, 4, 2, ctypes.byref(b))
    assert call(wsb=b.value - 1) == S.SFOC_E_WORKSPACE
    assert S.KERNEL_NAMES[11] == "fast"
