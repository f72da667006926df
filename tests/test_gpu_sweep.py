"""Reduced noise-sensitivity sweep on the GPU (3 pairs, 3 levels per noise
type): CMR is high without noise and does not rise with noise, for SFOC and
F-SFOC; the figures are printed."""
import sys

import pytest

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import sweep as W
from paper_2202_13347_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_reduced_sweep():
    assert torch.cuda.is_available()
    S.lib()
    rec = dict(synth.SWEEP, gaussian=[0.0, 0.005, 0.01], speckle=[0.0, 0.05, 0.1])
    res = W.run(3, rec, log=lambda s: print(s, file=sys.stderr, flush=True))
    for kind in ("gaussian", "speckle"):
        for k, vals in res[kind]["pooled_cmr"].items():
            assert vals[0] >= 0.9, (kind, k, vals)
            assert vals[-1] <= vals[0] + 0.02, (kind, k, vals)
