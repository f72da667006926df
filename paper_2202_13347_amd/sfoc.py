"""Thin Python binding of libsfoc.so (ctypes).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
If the library has not been built, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfoc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sfoc.h")

SFOC_OK, SFOC_E_INVALID_ARG, SFOC_E_UNSUPPORTED, SFOC_E_WORKSPACE, SFOC_E_HIP = 0, -1, -2, -3, -4
DTYPE_F32, DTYPE_BF16, DTYPE_F16 = 0, 1, 2
VALID, OOB, FLAT_T, FLAT_S, EDGE_PEAK, INCONSISTENT, LEARNED, NONFINITE = 1, 2, 4, 8, 16, 32, 64, 128


class SfocError(RuntimeError):
    """A library call returned a status other than SFOC_OK."""

    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class Params(ctypes.Structure):
    """sfoc_params: the SFOC filter bank (Section 3.1.2) and descriptor
    options, field for field as include/sfoc.h lays it out."""
    _fields_ = [("n_orient", ctypes.c_int32), ("n_s1", ctypes.c_int32), ("s1", ctypes.c_double * 8),
                ("n_s2", ctypes.c_int32), ("n_dil", ctypes.c_int32), ("s2", ctypes.c_double * 8),
                ("trunc", ctypes.c_double), ("sd1", ctypes.c_double), ("sd2", ctypes.c_double),
                ("eps", ctypes.c_double), ("K", ctypes.c_int32), ("dil", ctypes.c_int32 * 4),
                ("rectify", ctypes.c_int32), ("second_order", ctypes.c_int32), ("desc_dtype", ctypes.c_int32)]

    @property
    def z(self) -> int:
        return self.n_orient * (2 if self.second_order else 1)

    def copy(self) -> "Params":
        q = Params()
        ctypes.pointer(q)[0] = self
        return q


CP_DTYPE = np.dtype([("sen_row", np.int32), ("sen_col", np.int32), ("dy", np.int32), ("dx", np.int32),
                     ("sub_dy", np.float32), ("sub_dx", np.float32), ("score", np.float32),
                     ("flags", np.uint32)])
assert CP_DTYPE.itemsize == 32


class Pair(ctypes.Structure):
    """One image pair of a batched plan (device pointers)."""
    _fields_ = [("ref", ctypes.c_void_p), ("Hr", ctypes.c_int64), ("Wr", ctypes.c_int64), ("ldr", ctypes.c_int64),
                ("sen", ctypes.c_void_p), ("Hs", ctypes.c_int64), ("Ws", ctypes.c_int64), ("lds", ctypes.c_int64),
                ("ips", ctypes.c_void_p), ("prior", ctypes.c_void_p), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("r", ctypes.c_int32), ("fft_side", ctypes.c_int32), ("ncc", ctypes.c_void_p),
                ("cps", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    """sfoc_plan_info: what a batched plan decided (work items, tuned and
    cached shape classes, graph and persistent launches, the describe launch
    configuration, device bytes)."""
    _fields_ = [("n_pairs", ctypes.c_int32), ("describe_tiles", ctypes.c_int32),
                ("match_items", ctypes.c_int32 * 4), ("peak_items", ctypes.c_int32),
                ("tuned_classes", ctypes.c_int32), ("cached_classes", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("persistent", ctypes.c_int32 * 4), ("describe_config", ctypes.c_int32),
                ("direct_items", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


PLAN_GRAPH, PLAN_AUTOTUNE, PLAN_DENSE_SEN, PLAN_PERSISTENT, PLAN_DESCRIBE_ALT = 1, 2, 4, 8, 16
MATCH_DIRECT = 1   # fft_side naming the direct form (matrix cores; BF16/FP16, 2r+1 <= 32, m <= 64)


class RansacParams(ctypes.Structure):
    """sfoc_ransac_params: model kind, hypotheses, refinement passes, inlier
    threshold in pixels and the two image sizes (Section 3.2.3)."""
    _fields_ = [("model", ctypes.c_int32), ("n_hyp", ctypes.c_int32), ("n_refine", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("threshold", ctypes.c_double), ("Hs", ctypes.c_int32),
                ("Ws", ctypes.c_int32), ("Hr", ctypes.c_int32), ("Wr", ctypes.c_int32)]


MODEL_AFFINE, MODEL_PROJECTIVE = 6, 8
MODEL_SAMPLE = {MODEL_AFFINE: 3, MODEL_PROJECTIVE: 4}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded C-ABI library with its argument types set (loaded once;
    raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_13347_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER(Params)
        L.sfoc_status_string.restype = ctypes.c_char_p
        L.sfoc_status_string.argtypes = [ctypes.c_int]
        L.sfoc_params_preset.argtypes = [i32, P]
        L.sfoc_params_check.argtypes = [P, ctypes.POINTER(i32)]
        L.sfoc_describe_workspace.argtypes = [i64, i64, P, ctypes.POINTER(sz)]
        L.sfoc_describe.argtypes = [vp, i64, i64, i64, P, vp, vp, vp, vp, sz, vp]
        L.sfoc_describe_noalloc.argtypes = [vp, i64, i64, i64, P, vp, vp, vp, vp]
        L.sfoc_match_workspace.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.sfoc_match_window_workspace.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.sfoc_fastncc_match.argtypes = [vp, i64, i64, vp, i64, i64, vp, vp, i32, i32, vp, vp, i32, i32, i32,
                                         vp, vp, vp, sz, vp]
        L.sfoc_register_workspace.argtypes = [i64, i64, i64, i64, i32, i32, i32, P, ctypes.POINTER(sz)]
        L.sfoc_register_cps.argtypes = [vp, i64, i64, i64, vp, i64, i64, i64, vp, vp, i32, i32, i32, P,
                                        vp, vp, vp, sz, vp]
        L.sfoc_register_streamed_workspace.argtypes = [i64, i64, i64, i64, i32, i32, i32, i32, i32, P,
                                                       ctypes.POINTER(sz)]
        L.sfoc_register_cps_streamed.argtypes = [vp, i64, i64, i64, vp, i64, i64, i64, vp, vp, i32, i32, i32, i32,
                                                 i32, P, vp, vp, vp, sz, vp]
        L.sfoc_plan_create.argtypes = [ctypes.POINTER(Pair), i32, P, i32, ctypes.c_char_p, vp,
                                       ctypes.POINTER(vp)]
        L.sfoc_register_cps_batched.argtypes = [vp, vp]
        L.sfoc_plan_destroy.argtypes = [vp]
        L.sfoc_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                         i32]
        L.sfoc_match_candidates.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), i32]
        L.sfoc_sensed_tiles.argtypes = [vp, vp, i32, i32, i32, i64, i64, i64, i64, i32, vp, i64]
        L.sfoc_sensed_tiles.restype = i64
        f32p = ctypes.c_void_p
        L.sfoc_head_features.argtypes = [vp, i64, i64, vp, vp, i64, i64, i32, i32, vp, vp, i32, i32, i32, vp, vp,
                                         vp, vp, vp]
        L.sfoc_head_workspace.argtypes = [i32, i32, ctypes.POINTER(sz)]
        L.sfoc_head_forward.argtypes = [vp, vp, vp, i32, vp, vp, sz, vp]
        L.sfoc_head_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, vp, i32, vp, vp, vp, sz,
                                           vp]
        L.sfoc_head_infer.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, sz, vp]
        L.sfoc_ransac_workspace.argtypes = [i32, ctypes.POINTER(RansacParams), ctypes.POINTER(sz)]
        L.sfoc_ransac_cps.argtypes = [vp, vp, i32, vp, ctypes.POINTER(RansacParams), vp, sz, vp, vp, vp, vp, vp]
        L.sfoc_rectify.argtypes = [vp, i64, i64, i64, vp, vp, i64, i64, i64, ctypes.c_float, vp]
        L.sfoc_fast_workspace.argtypes = [i64, i64, i32, i32, i32, ctypes.POINTER(sz)]
        L.sfoc_detect_ips.argtypes = [vp, i64, i64, i64, ctypes.c_float, i32, i32, i32, i32, vp, vp, vp, vp,
                                      vp, sz, vp]
        L.sfoc_trace_enable.argtypes = [ctypes.c_int]
        L.sfoc_trace_collect.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int]
        for name in ("sfoc_trace_enable", "sfoc_trace_collect", "sfoc_params_preset", "sfoc_params_check", "sfoc_describe_workspace", "sfoc_describe",
                     "sfoc_match_workspace", "sfoc_fastncc_match", "sfoc_register_workspace",
                     "sfoc_register_cps", "sfoc_register_streamed_workspace", "sfoc_register_cps_streamed", "sfoc_plan_create", "sfoc_register_cps_batched", "sfoc_plan_destroy",
                     "sfoc_plan_get_info", "sfoc_match_candidates", "sfoc_head_features", "sfoc_head_workspace",
                     "sfoc_head_forward", "sfoc_head_train_step", "sfoc_head_infer", "sfoc_ransac_workspace",
                     "sfoc_ransac_cps", "sfoc_rectify", "sfoc_fast_workspace", "sfoc_detect_ips"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/sfoc.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sfoc_[a-z0-9_]+)\s*\(", txt)))


def status_string(s: int) -> str:
    """Text of a library status code."""
    return lib().sfoc_status_string(int(s)).decode()


def _check(rc: int, what: str):
    if rc != SFOC_OK:
        raise SfocError(rc, what)


def preset(which: str | int = "baseline", dtype: int = DTYPE_F32) -> Params:
    """'paper' (N=6; sigma 0.6/0.8/1.0 and 1.5) or 'baseline' (N=8; 1/2/3)."""
    w = {"paper": 0, "baseline": 1}.get(which, which)
    p = Params()
    _check(lib().sfoc_params_preset(int(w), ctypes.byref(p)), "sfoc_params_preset")
    p.desc_dtype = dtype
    return p


def params(n_orient=8, s1=(1.0, 2.0, 3.0), s2=(1.0, 2.0, 3.0), trunc=3.0, sd1=1.0, sd2=1.5, K=1,
           dil=(1, 2, 3), eps=1e-8, rectify=0, second_order=True, dtype=DTYPE_F32) -> Params:
    """A Params from explicit values: orientations, first- and second-order
    scales, truncation, the two smoothing deviations, K, dilations, the
    rectification mode (abs / signed / relu) and the descriptor dtype."""
    p = Params()
    p.n_orient = n_orient
    p.n_s1 = len(s1)
    for i, v in enumerate(s1):
        p.s1[i] = v
    p.n_s2 = len(s2)
    for i, v in enumerate(s2):
        p.s2[i] = v
    p.trunc, p.sd1, p.sd2, p.eps, p.K = trunc, sd1, sd2, eps, K
    p.n_dil = len(dil)
    for i, v in enumerate(dil):
        p.dil[i] = v
    p.rectify = {"abs": 0, "signed": 1, "relu": 2}.get(rectify, rectify)
    p.second_order = int(bool(second_order))
    p.desc_dtype = dtype
    return p


def check_params(p: Params) -> int:
    """Validates p in the library and returns its descriptor depth z."""
    z = ctypes.c_int32(0)
    _check(lib().sfoc_params_check(ctypes.byref(p), ctypes.byref(z)), "sfoc_params_check")
    return z.value


# ---------------------------------------------------------------- device --
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _desc_torch_dtype(dt: int):
    torch = _torch()
    return {DTYPE_F32: torch.float32, DTYPE_BF16: torch.bfloat16, DTYPE_F16: torch.float16}[dt]


def describe_workspace(H: int, W: int, p: Params) -> int:
    """Bytes of scratch sfoc_describe needs for an (H, W) image."""
    b = ctypes.c_size_t(0)
    _check(lib().sfoc_describe_workspace(H, W, ctypes.byref(p), ctypes.byref(b)), "sfoc_describe_workspace")
    return b.value


def describe(img, p: Params, integrals: bool = True, stream=None, out=None):
    """SFOC of one float32 (H, W) CUDA image.  Returns (desc (z, H, W),
    integ1, integ2) (the integral images are None if not requested)."""
    torch = _torch()
    assert img.is_cuda and img.dtype == torch.float32 and img.dim() == 2 and img.stride(1) == 1
    H, W = img.shape
    z = check_params(p)
    desc = out if out is not None else torch.empty((z, H, W), dtype=_desc_torch_dtype(p.desc_dtype),
                                                   device=img.device)
    i1 = i2 = ws = None
    wsb = 0
    if integrals:
        i1 = torch.empty((H + 1, W + 1), dtype=torch.float64, device=img.device)
        i2 = torch.empty_like(i1)
        wsb = describe_workspace(H, W, p)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=img.device)
    rc = lib().sfoc_describe(_ptr(img), H, W, img.stride(0), ctypes.byref(p), _ptr(desc), _ptr(i1), _ptr(i2),
                             _ptr(ws), wsb, _stream(stream))
    _check(rc, "sfoc_describe")
    return desc, i1, i2


NOALLOC_SCRATCH_BYTES = 64 << 20   # SFOC_NOALLOC_SCRATCH_BYTES


def describe_noalloc(img, p: Params, desc, integ1, integ2, stream=None):
    """sfoc_describe_noalloc into caller-provided outputs (desc (z, H, W),
    integ1 and integ2 (H+1, W+1) float64 CUDA tensors): the library
    allocates nothing for it."""
    H, W = img.shape
    rc = lib().sfoc_describe_noalloc(_ptr(img), H, W, img.stride(0), ctypes.byref(p), _ptr(desc), _ptr(integ1),
                                     _ptr(integ2), _stream(stream))
    _check(rc, "sfoc_describe_noalloc")
    return desc, integ1, integ2


def fastncc_match(desc_sen, desc_ref, integ1, integ2, ips, m: int, r: int, prior=None, want_ncc=False,
                  stream=None):
    """CPs (an (n, 8) int32 CUDA tensor of 32-byte records) and optionally
    the NCC surfaces (n, 2r+1, 2r+1).  integ1 = integ2 = None: the integral
    images are built per search window (in the workspace)."""
    torch = _torch()
    z, Hs, Ws = desc_sen.shape
    _, Hr, Wr = desc_ref.shape
    dt = {torch.float32: DTYPE_F32, torch.bfloat16: DTYPE_BF16, torch.float16: DTYPE_F16}[desc_sen.dtype]
    n = ips.shape[0]
    V = 2 * r + 1
    cps = torch.empty((n, 8), dtype=torch.int32, device=desc_sen.device)
    ncc = torch.empty((n, V, V), dtype=torch.float32, device=desc_sen.device) if want_ncc else None
    b = ctypes.c_size_t(0)
    query = lib().sfoc_match_workspace if integ1 is not None else lib().sfoc_match_window_workspace
    _check(query(n, m, r, z, ctypes.byref(b)), "match workspace query")
    ws = torch.empty(b.value, dtype=torch.uint8, device=desc_sen.device) if b.value else None
    rc = lib().sfoc_fastncc_match(_ptr(desc_sen), Hs, Ws, _ptr(desc_ref), Hr, Wr, _ptr(integ1), _ptr(integ2),
                                  z, dt, _ptr(ips), _ptr(prior), n, m, r, _ptr(ncc), _ptr(cps), _ptr(ws), b.value,
                                  _stream(stream))
    _check(rc, "sfoc_fastncc_match")
    return (cps, ncc) if want_ncc else cps


def register_workspace(Hr, Wr, Hs, Ws, n, m, r, p: Params) -> int:
    """Bytes of scratch sfoc_register_cps needs for these sizes."""
    b = ctypes.c_size_t(0)
    _check(lib().sfoc_register_workspace(Hr, Wr, Hs, Ws, n, m, r, ctypes.byref(p), ctypes.byref(b)),
           "sfoc_register_workspace")
    return b.value


class Registrar:
    """Holds the workspace of sfoc_register_cps for one shape, so repeated
    calls allocate nothing."""

    def __init__(self, Hr, Wr, Hs, Ws, n, m, r, p: Params, device="cuda", want_ncc=False):
        torch = _torch()
        self.p = p.copy()
        self.shape = (Hr, Wr, Hs, Ws, n, m, r)
        self.wsb = register_workspace(Hr, Wr, Hs, Ws, n, m, r, self.p)
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=device)
        self.cps = torch.empty((n, 8), dtype=torch.int32, device=device)
        V = 2 * r + 1
        self.ncc = torch.empty((n, V, V), dtype=torch.float32, device=device) if want_ncc else None

    def __call__(self, ref, sen, ips, prior=None, stream=None):
        Hr, Wr, Hs, Ws, n, m, r = self.shape
        assert ref.shape == (Hr, Wr) and sen.shape == (Hs, Ws) and ips.shape[0] == n
        rc = lib().sfoc_register_cps(_ptr(ref), Hr, Wr, ref.stride(0), _ptr(sen), Hs, Ws, sen.stride(0),
                                     _ptr(ips), _ptr(prior), n, m, r, ctypes.byref(self.p), _ptr(self.ncc),
                                     _ptr(self.cps), _ptr(self.ws), self.wsb, _stream(stream))
        _check(rc, "sfoc_register_cps")
        return self.cps


def register_cps(ref, sen, ips, m: int, r: int, p: Params, prior=None, want_ncc=False, stream=None):
    """One-shot describe + Fast-NCC matching of a pair (allocates its own
    workspace; Registrar reuses one).  Returns the CPs, and the NCC
    surfaces when want_ncc."""
    R = Registrar(ref.shape[0], ref.shape[1], sen.shape[0], sen.shape[1], ips.shape[0], m, r, p,
                  device=ref.device, want_ncc=want_ncc)
    cps = R(ref, sen, ips, prior, stream)
    return (cps, R.ncc) if want_ncc else cps


class StreamedRegistrar:
    """Holds the one-band workspace of sfoc_register_cps_streamed: IPs sorted
    by row, taken band_rows rows at a time, row priors within max_prior."""

    def __init__(self, Hr, Wr, Hs, Ws, n, m, r, p: Params, band_rows: int, max_prior: int = 0, device="cuda",
                 want_ncc=False):
        torch = _torch()
        self.p = p.copy()
        self.shape = (Hr, Wr, Hs, Ws, n, m, r)
        self.band_rows, self.max_prior = int(band_rows), int(max_prior)
        b = ctypes.c_size_t(0)
        _check(lib().sfoc_register_streamed_workspace(Hr, Wr, Hs, Ws, n, m, r, self.band_rows, self.max_prior,
                                                      ctypes.byref(self.p), ctypes.byref(b)),
               "sfoc_register_streamed_workspace")
        self.wsb = b.value
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=device)
        self.cps = torch.empty((n, 8), dtype=torch.int32, device=device)
        V = 2 * r + 1
        self.ncc = torch.empty((n, V, V), dtype=torch.float32, device=device) if want_ncc else None

    def __call__(self, ref, sen, ips, prior=None, stream=None):
        Hr, Wr, Hs, Ws, n, m, r = self.shape
        assert ref.shape == (Hr, Wr) and sen.shape == (Hs, Ws) and ips.shape[0] == n
        rc = lib().sfoc_register_cps_streamed(_ptr(ref), Hr, Wr, ref.stride(0), _ptr(sen), Hs, Ws, sen.stride(0),
                                              _ptr(ips), _ptr(prior), n, m, r, self.band_rows, self.max_prior,
                                              ctypes.byref(self.p), _ptr(self.ncc), _ptr(self.cps), _ptr(self.ws),
                                              self.wsb, _stream(stream))
        _check(rc, "sfoc_register_cps_streamed")
        return self.cps


class Plan:
    """A batched plan over image pairs (sfoc_plan_create).

    pairs: sequence of dicts with CUDA tensors ref (Hr, Wr) float32, sen
    (Hs, Ws) float32, ips (n, 2) int32, optional prior (n, 2) int32, and ints
    m, r, optional fft_side (0 / 64 / 128 / 160 / 192, or MATCH_DIRECT).  The plan owns per-pair outputs
    cps (n, 8) int32 and, with want_ncc, ncc (n, 2r+1, 2r+1); it keeps
    references to every input tensor for its lifetime.  Calling the plan
    runs sfoc_register_cps_batched on the current stream."""

    def __init__(self, pairs, p: Params, flags: int = 0, tune_cache: str | None = None, want_ncc=False,
                 stream=None):
        torch = _torch()
        self.p = p.copy()
        self.inputs = []
        self.cps, self.ncc = [], []
        arr = (Pair * len(pairs))()
        for k, q in enumerate(pairs):
            ref, sen, ips = q["ref"], q["sen"], q["ips"]
            prior = q.get("prior")
            for t in (ref, sen):
                assert t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.stride(1) == 1
            assert ips.dtype == torch.int32 and ips.is_contiguous()
            n, m, r = ips.shape[0], int(q["m"]), int(q["r"])
            cps = torch.empty((n, 8), dtype=torch.int32, device=ref.device)
            V = 2 * r + 1
            ncc = torch.empty((n, V, V), dtype=torch.float32, device=ref.device) if want_ncc else None
            self.inputs.append((ref, sen, ips, prior))
            self.cps.append(cps)
            self.ncc.append(ncc)
            a = arr[k]
            a.ref, a.Hr, a.Wr, a.ldr = ref.data_ptr(), ref.shape[0], ref.shape[1], ref.stride(0)
            a.sen, a.Hs, a.Ws, a.lds = sen.data_ptr(), sen.shape[0], sen.shape[1], sen.stride(0)
            a.ips = ips.data_ptr()
            a.prior = prior.data_ptr() if prior is not None else None
            a.n, a.m, a.r, a.fft_side = n, m, r, int(q.get("fft_side", 0))
            a.ncc = ncc.data_ptr() if ncc is not None else None
            a.cps = cps.data_ptr()
        self._pairs = arr
        h = ctypes.c_void_p(0)
        tc = tune_cache.encode() if tune_cache else None
        _check(lib().sfoc_plan_create(arr, len(pairs), ctypes.byref(self.p), flags, tc, _stream(stream),
                                      ctypes.byref(h)), "sfoc_plan_create")
        self.handle = h

    def __call__(self, stream=None):
        _check(lib().sfoc_register_cps_batched(self.handle, _stream(stream)), "sfoc_register_cps_batched")
        return self.cps

    def info(self) -> dict:
        n = len(self.cps)
        inf = PlanInfo()
        L = (ctypes.c_int32 * n)()
        nb = (ctypes.c_int32 * n)()
        _check(lib().sfoc_plan_get_info(self.handle, ctypes.byref(inf), L, nb, n), "sfoc_plan_get_info")
        return {"n_pairs": inf.n_pairs, "describe_tiles": inf.describe_tiles,
                "match_items": tuple(inf.match_items), "peak_items": inf.peak_items,
                "tuned_classes": inf.tuned_classes, "cached_classes": inf.cached_classes, "graph": inf.graph,
                "persistent": tuple(inf.persistent), "describe_config": inf.describe_config,
                "direct_items": inf.direct_items,
                "device_bytes": inf.device_bytes, "fft_side": list(L), "blocks": list(nb)}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().sfoc_plan_destroy(self.handle), "sfoc_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def match_candidates(m: int, r: int) -> list[tuple[int, int]]:
    """[(transform side, offset blocks per axis)] an autotuner may time."""
    L = (ctypes.c_int32 * 4)()
    nb = (ctypes.c_int32 * 4)()
    k = lib().sfoc_match_candidates(m, r, L, nb, 4)
    if k < 0:
        raise SfocError(k, "sfoc_match_candidates")
    return [(L[i], nb[i]) for i in range(k)]


COVER_TEMPLATE, COVER_GRID, COVER_SMALLER = 0, 1, 2


def sensed_tiles(ips: np.ndarray, m: int, r: int, Hs: int, Ws: int, Hr: int, Wr: int, prior=None,
                 cover: int = COVER_TEMPLATE) -> np.ndarray:
    """(k, 2) int32 (row, column) origins of the distinct 32 x 32
    sensed-image tiles over the templates of the in-bounds IPs (host
    arrays, no device work): COVER_TEMPLATE, each IP's template-aligned
    tiles (the pair call); COVER_GRID, the image-grid tiles the templates
    touch; COVER_SMALLER, the shorter list (sparse plans)."""
    ips = np.ascontiguousarray(ips, dtype=np.int32).reshape(-1, 2)
    pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.int32)
    k = (m + 31) // 32
    cap = len(ips) * max(k * (k + 1), (k + 1) * (k + 1))
    out = np.zeros((cap, 2), dtype=np.int32)
    c = lib().sfoc_sensed_tiles(ips.ctypes.data, None if pr is None else pr.ctypes.data, len(ips), m, r, Hs, Ws,
                                Hr, Wr, cover, out.ctypes.data if cap else None, cap)
    if c < 0:
        raise SfocError(int(c), "sfoc_sensed_tiles")
    return out[:c]


HEAD_PARAMS, HEAD_CROP, HEAD_NSTAT = 54051, 33, 8


def head_features(desc_sen, desc_ref, integ1, integ2, ips, m: int, r: int, ncc, cps, prior=None, stream=None):
    """(crops (n, 33, 33), stats (n, 8)) float32 CUDA tensors for the head."""
    torch = _torch()
    z, Hs, Ws = desc_sen.shape
    _, Hr, Wr = desc_ref.shape
    dt = {torch.float32: DTYPE_F32, torch.bfloat16: DTYPE_BF16, torch.float16: DTYPE_F16}[desc_sen.dtype]
    n = ips.shape[0]
    crops = torch.empty((n, HEAD_CROP, HEAD_CROP), dtype=torch.float32, device=desc_sen.device)
    stats = torch.empty((n, HEAD_NSTAT), dtype=torch.float32, device=desc_sen.device)
    rc = lib().sfoc_head_features(_ptr(desc_sen), Hs, Ws, _ptr(integ1), _ptr(integ2), Hr, Wr, z, dt, _ptr(ips),
                                  _ptr(prior), n, m, r, _ptr(ncc), _ptr(cps), _ptr(crops), _ptr(stats),
                                  _stream(stream))
    _check(rc, "sfoc_head_features")
    return crops, stats


def head_workspace(n: int, train: bool) -> int:
    """Bytes of scratch the learned head needs for n CPs (more when
    training, for the saved activations)."""
    b = ctypes.c_size_t(0)
    _check(lib().sfoc_head_workspace(n, int(train), ctypes.byref(b)), "sfoc_head_workspace")
    return b.value


class Head:
    """Parameters (float32 master copy), Adam moments and workspaces of the
    learned head on one device.  Every computation runs in the library."""

    def __init__(self, params, device="cuda"):
        torch = _torch()
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        assert p.numel() == HEAD_PARAMS
        self.params = p.to(device).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.device = device
        self._ws = {}

    def _workspace(self, n, train):
        torch = _torch()
        key = (n, bool(train))
        if key not in self._ws:
            self._ws = {k: w for k, w in self._ws.items() if k[1] != bool(train)}   # one per mode
            self._ws[key] = torch.empty(max(1, head_workspace(n, train)), dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def forward(self, crops, stats, stream=None):
        torch = _torch()
        n = crops.shape[0]
        out = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        if n:
            ws = self._workspace(n, False)
            _check(lib().sfoc_head_forward(_ptr(self.params), _ptr(crops), _ptr(stats), n, _ptr(out), _ptr(ws),
                                           ws.numel(), _stream(stream)), "sfoc_head_forward")
        return out

    def train_step(self, crops, stats, label, target, lr: float, want_grad=False, stream=None):
        """One Adam step; returns (loss tensor (1,), gradient or None)."""
        torch = _torch()
        n = crops.shape[0]
        ws = self._workspace(n, True)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(HEAD_PARAMS, dtype=torch.float32, device=self.device) if want_grad else None
        self.t += 1
        _check(lib().sfoc_head_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.t, float(lr),
                                          _ptr(crops), _ptr(stats), _ptr(label), _ptr(target), n, _ptr(grad),
                                          _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)),
               "sfoc_head_train_step")
        return loss, grad

    def infer(self, crops, stats, cps, threshold: float = 0.5, want_out=False, stream=None):
        """Applies the head to CP records in place (eligible CPs only)."""
        torch = _torch()
        n = crops.shape[0]
        out = torch.empty((n, 3), dtype=torch.float32, device=self.device) if want_out else None
        if n:
            ws = self._workspace(n, False)
            _check(lib().sfoc_head_infer(_ptr(self.params), _ptr(crops), _ptr(stats), n, float(threshold), _ptr(cps),
                                         _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "sfoc_head_infer")
        return out


KERNEL_NAMES = ("describe", "integral", "match", "consistency", "peak", "head_features", "head_forward",
                "head_backward", "head_adam", "ransac", "rectify", "fast")


def ransac_params(model: int, n_hyp: int, sizes, threshold: float = 1.5, n_refine: int = 2) -> RansacParams:
    """sizes = (Hs, Ws, Hr, Wr)."""
    Hs, Ws, Hr, Wr = (int(v) for v in sizes)
    return RansacParams(int(model), int(n_hyp), int(n_refine), 0, float(threshold), Hs, Ws, Hr, Wr)


def ransac_workspace(n: int, rp: RansacParams) -> int:
    """Bytes of scratch sfoc_ransac_cps needs for n CPs."""
    b = ctypes.c_size_t(0)
    _check(lib().sfoc_ransac_workspace(int(n), ctypes.byref(rp), ctypes.byref(b)), "sfoc_ransac_workspace")
    return b.value


class Ransac:
    """sfoc_ransac_cps with its workspace and outputs allocated once, for n
    CPs and the given parameters.  Calling it updates the CP flags in place
    and returns the device tensors (model (9,) float64, info (4,) int32)."""

    def __init__(self, n: int, rp: RansacParams, device="cuda"):
        torch = _torch()
        self.n, self.rp = int(n), rp
        self.k = MODEL_SAMPLE[rp.model]
        self.ws = torch.empty(ransac_workspace(n, rp), dtype=torch.uint8, device=device)
        self.model = torch.zeros(9, dtype=torch.float64, device=device)
        self.info = torch.zeros(4, dtype=torch.int32, device=device)

    def __call__(self, cps, words, prior=None, counts=None, hyp_models=None, stream=None):
        if cps.shape[0] != self.n:
            raise ValueError(f"{cps.shape[0]} CPs, plan for {self.n}")
        if words.numel() != self.rp.n_hyp * self.k or words.element_size() != 4 or not words.is_contiguous():
            raise ValueError("words: n_hyp * k contiguous 32-bit values")
        _check(lib().sfoc_ransac_cps(_ptr(cps), _ptr(prior), self.n, _ptr(words), ctypes.byref(self.rp),
                                     _ptr(self.ws), self.ws.numel(), _ptr(self.model), _ptr(self.info),
                                     _ptr(counts), _ptr(hyp_models), _stream(stream)), "sfoc_ransac_cps")
        return self.model, self.info


def ransac(cps, words, model: int, sizes, threshold: float = 1.5, n_refine: int = 2, prior=None,
           want_counts: bool = False, want_models: bool = False, stream=None) -> dict:
    """RANSAC over the CPs of one pair (device tensor (n, 8) int32, updated
    in place).  words: device tensor of n_hyp * k 32-bit random words
    (int32 holding the uint32 bit patterns).  Synchronises and returns host
    values: model (3x3, pixels), n_cand, inliers, best, status, and the
    per-hypothesis counts / minimal models when asked for."""
    torch = _torch()
    k = MODEL_SAMPLE[model]
    n_hyp = words.numel() // k
    rp = ransac_params(model, n_hyp, sizes, threshold, n_refine)
    R = Ransac(cps.shape[0], rp, device=words.device)
    counts = torch.full((n_hyp,), -2, dtype=torch.int32, device=words.device) if want_counts else None
    hyp = torch.zeros((n_hyp, 9), dtype=torch.float64, device=words.device) if want_models else None
    m, info = R(cps, words, prior=prior, counts=counts, hyp_models=hyp, stream=stream)
    info = info.cpu().numpy()
    out = dict(model=m.cpu().numpy().reshape(3, 3), n_cand=int(info[0]), inliers=int(info[1]), best=int(info[2]),
               status=int(info[3]))
    if want_counts:
        out["counts"] = counts.cpu().numpy()
    if want_models:
        out["hyp_models"] = hyp.cpu().numpy().reshape(-1, 3, 3)
    return out


def rectify(sen, model, out_shape, fill: float = 0.0, out=None, stream=None):
    """Resample the sensed image (Hs x Ws float32 device tensor, rows may be
    padded) into an out_shape reference grid through the sensed -> reference
    model (device float64 tensor of 9, e.g. Ransac.model, or a host 3x3)."""
    torch = _torch()
    Ho, Wo = (int(v) for v in out_shape)
    if not torch.is_tensor(model):
        model = torch.from_numpy(np.ascontiguousarray(model, np.float64).reshape(9)).to(sen.device)
    if model.dtype != torch.float64 or model.numel() != 9 or not model.is_contiguous():
        raise ValueError("model: 9 contiguous float64 values")
    if sen.dtype != torch.float32 or sen.dim() != 2 or sen.stride(1) != 1:
        raise ValueError("sen: 2-D float32 with unit column stride")
    if out is None:
        out = torch.empty((Ho, Wo), dtype=torch.float32, device=sen.device)
    _check(lib().sfoc_rectify(_ptr(sen), sen.shape[0], sen.shape[1], sen.stride(0), _ptr(model), _ptr(out), Ho, Wo,
                              out.stride(0), float(fill), _stream(stream)), "sfoc_rectify")
    return out


def fast_workspace(H: int, W: int, nby: int, nbx: int, per_block: int) -> int:
    """Bytes of scratch sfoc_detect_ips needs for this image and block layout."""
    b = ctypes.c_size_t(0)
    _check(lib().sfoc_fast_workspace(int(H), int(W), int(nby), int(nbx), int(per_block), ctypes.byref(b)),
           "sfoc_fast_workspace")
    return b.value


class Detector:
    """sfoc_detect_ips with its workspace and outputs allocated once for one
    image size and block layout.  Calling it returns the device tensors
    (ips (capacity, 2) int32, scores, counts, n_out); the first n_out rows of
    ips are the interest points."""

    def __init__(self, H: int, W: int, nby: int, nbx: int, per_block: int, threshold: float, margin: int,
                 device="cuda"):
        torch = _torch()
        self.shape = (int(H), int(W))
        self.nby, self.nbx, self.per = int(nby), int(nbx), int(per_block)
        self.threshold, self.margin = float(threshold), int(margin)
        cap = self.nby * self.nbx * self.per
        self.ws = torch.empty(fast_workspace(H, W, nby, nbx, per_block), dtype=torch.uint8, device=device)
        self.ips = torch.zeros((cap, 2), dtype=torch.int32, device=device)
        self.scores = torch.zeros(cap, dtype=torch.float32, device=device)
        self.counts = torch.zeros(self.nby * self.nbx, dtype=torch.int32, device=device)
        self.n_out = torch.zeros(1, dtype=torch.int32, device=device)

    def __call__(self, img, stream=None):
        if tuple(img.shape) != self.shape or img.dtype != _torch().float32 or img.stride(1) != 1:
            raise ValueError("img: the detector's (H, W) float32 with unit column stride")
        _check(lib().sfoc_detect_ips(_ptr(img), self.shape[0], self.shape[1], img.stride(0), self.threshold,
                                     self.margin, self.nby, self.nbx, self.per, _ptr(self.ips), _ptr(self.scores),
                                     _ptr(self.counts), _ptr(self.n_out), _ptr(self.ws), self.ws.numel(),
                                     _stream(stream)), "sfoc_detect_ips")
        return self.ips, self.scores, self.counts, self.n_out


def detect_ips(img, threshold: float, margin: int, nby: int, nbx: int, per_block: int = 1, stream=None):
    """Block-based FAST on a device image; synchronises and returns the
    interest points as a device tensor (n, 2) int32, with the host scores
    and per-block counts."""
    D = Detector(img.shape[0], img.shape[1], nby, nbx, per_block, threshold, margin, device=img.device)
    ips, sc, cnt, n = D(img, stream)
    k = int(n.item())
    return ips[:k].clone(), sc[:k].cpu().numpy(), cnt.cpu().numpy()


def trace_enable(on: bool = True):
    """Switches the per-kernel event timing of the library on or off."""
    _check(lib().sfoc_trace_enable(int(on)), "sfoc_trace_enable")


def trace_collect() -> dict:
    """{kernel: (total ms, launches)} since the last collection."""
    n = len(KERNEL_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    rc = lib().sfoc_trace_collect(ms, cnt, n)
    if rc < 0:
        raise SfocError(rc, "sfoc_trace_collect")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_NAMES)}


def cps_to_numpy(cps) -> np.ndarray:
    """(n, 8) int32 tensor or array of records -> structured array."""
    a = cps.detach().cpu().numpy() if hasattr(cps, "detach") else np.asarray(cps)
    return np.ascontiguousarray(a, dtype=np.int32).view(CP_DTYPE).reshape(-1)
