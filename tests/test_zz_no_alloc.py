"""sfoc_describe_noalloc (through the C ABI): the no-allocation variant of
sfoc_describe with integral images gives sfoc_describe's results bit for bit
on two calls in a row, the second with a smaller image (the library-owned
aggregate array keeps the first call's contents), and rejects images whose
aggregates exceed the array before launching anything."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _outputs(H, W, p):
    z = S.check_params(p)
    dt = {S.DTYPE_F32: torch.float32, S.DTYPE_BF16: torch.bfloat16, S.DTYPE_F16: torch.float16}[p.desc_dtype]
    d = torch.full((z, H, W), float("nan"), dtype=dt, device="cuda")
    i1 = torch.full((H + 1, W + 1), float("nan"), dtype=torch.float64, device="cuda")
    return d, i1, torch.full_like(i1, float("nan"))


@pytest.mark.parametrize("preset,dtype", [("baseline", S.DTYPE_F32), ("paper", S.DTYPE_BF16)])
def test_noalloc_equals_describe(preset, dtype):
    assert torch.cuda.is_available()
    S.lib()
    p = S.preset(preset, dtype=dtype)
    for k, (H, W) in enumerate([(700, 650), (130, 97)]):      # second call smaller
        say("noalloc", preset, dtype, "call", k, (H, W))
        img = torch.from_numpy(synth.make_pair(30 + k, (H, W), 2.0).sen).cuda()
        want = S.describe(img, p)
        got = S.describe_noalloc(img, p, *_outputs(H, W, p))
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            assert torch.equal(a, b)


def test_noalloc_rejects_oversize_and_bad_args():
    S.lib()
    p = S.preset("baseline")
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the calls fail their checks first
    big = 9000                       # aggregates above the library's array
    assert S.describe_workspace(big, big, p) > S.NOALLOC_SCRATCH_BYTES
    assert S.lib().sfoc_describe_noalloc(fake, big, big, big, ctypes.byref(p), fake, fake, fake, None) == \
        S.SFOC_E_UNSUPPORTED
    assert S.lib().sfoc_describe_noalloc(fake, 64, 64, 64, ctypes.byref(p), fake, None, fake, None) == \
        S.SFOC_E_INVALID_ARG
    assert S.lib().sfoc_describe_noalloc(fake, 64, 64, 32, ctypes.byref(p), fake, fake, fake, None) == \
        S.SFOC_E_INVALID_ARG
