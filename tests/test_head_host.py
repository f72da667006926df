"""Host-side checks of the head entry points: workspace sizes and argument
rejection before any device work."""
import ctypes

import pytest

from paper_2202_13347_amd import sfoc as S

F = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
L = None


def lib():
    return S.lib()


def test_workspace_sizes():
    a, b = S.head_workspace(16, False), S.head_workspace(32, False)
    assert 0 < a < b
    assert S.head_workspace(32, True) > b
    sz = ctypes.c_size_t(0)
    assert lib().sfoc_head_workspace(-1, 0, ctypes.byref(sz)) == S.SFOC_E_INVALID_ARG
    assert lib().sfoc_head_workspace(65537, 0, ctypes.byref(sz)) == S.SFOC_E_UNSUPPORTED
    assert lib().sfoc_head_workspace(65536, 1, ctypes.byref(sz)) == S.SFOC_OK


def test_train_step_rejects_bad_arguments():
    ws = S.head_workspace(8, True)
    f = lib().sfoc_head_train_step
    assert f(F, F, F, 0, 1e-3, F, F, F, F, 8, None, None, F, ws, None) == S.SFOC_E_INVALID_ARG   # t < 1
    assert f(F, F, F, 1, -1.0, F, F, F, F, 8, None, None, F, ws, None) == S.SFOC_E_INVALID_ARG   # lr < 0
    assert f(None, F, F, 1, 1e-3, F, F, F, F, 8, None, None, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert f(F, F, F, 1, 1e-3, F, F, None, F, 8, None, None, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert f(F, F, F, 1, 1e-3, F, F, F, F, 8, None, None, F, ws - 1, None) == S.SFOC_E_WORKSPACE
    assert f(F, F, F, 1, 1e-3, F, F, F, F, 70000, None, None, F, ws, None) == S.SFOC_E_UNSUPPORTED
    assert f(F, F, F, 1, 1e-3, F, F, F, F, 0, None, None, None, 0, None) == S.SFOC_OK


def test_forward_and_infer_reject_bad_arguments():
    ws = S.head_workspace(8, False)
    assert lib().sfoc_head_forward(F, F, F, 8, F, F, ws - 1, None) == S.SFOC_E_WORKSPACE
    assert lib().sfoc_head_forward(F, None, F, 8, F, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert lib().sfoc_head_forward(F, F, F, -1, F, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert lib().sfoc_head_infer(F, F, F, 8, 1.5, F, None, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert lib().sfoc_head_infer(F, F, F, 8, 0.5, None, None, F, ws, None) == S.SFOC_E_INVALID_ARG
    assert lib().sfoc_head_infer(F, F, F, 0, 0.5, None, None, None, 0, None) == S.SFOC_OK


def test_features_rejects_bad_arguments():
    f = lib().sfoc_head_features
    assert f(F, 64, 64, F, F, 64, 64, 16, 0, F, None, 4, 2, 4, F, F, F, F, None) == S.SFOC_E_INVALID_ARG  # m < 3
    assert f(F, 64, 64, F, F, 64, 64, 16, 7, F, None, 4, 16, 4, F, F, F, F, None) == S.SFOC_E_INVALID_ARG  # dtype
    assert f(F, 64, 64, None, F, 64, 64, 16, 0, F, None, 4, 16, 4, F, F, F, F, None) == S.SFOC_E_INVALID_ARG
    assert f(F, 64, 64, F, F, 64, 64, 16, 0, F, None, 4, 16, 4, None, F, F, F, None) == S.SFOC_E_INVALID_ARG
    assert f(None, 64, 64, None, None, 64, 64, 16, 0, None, None, 0, 16, 4, None, None, None, None, None) == S.SFOC_OK
