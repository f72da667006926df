"""Host pieces of the noise-sensitivity sweep (no GPU): the CMR count on
handcrafted CP records, and the noise generators' statistics (Gaussian:
mean 0, variance v; speckle: multiplicative, uniform, variance v) and
seeding."""
import numpy as np
import pytest

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import sweep as W
from paper_2202_13347_amd import synth


def test_cmr_counts():
    c = np.zeros(6, dtype=S.CP_DTYPE)
    shift = (3.3, -2.2)
    c["dy"] = [3, 3, 5, 3, 3, 0]
    c["dx"] = [-2, -2, -2, -2, 0, 0]
    c["sub_dy"] = [0.3, -0.4, 0.3, 0.3, 0.3, 0.0]
    c["sub_dx"] = [-0.2, 0.1, -0.2, -0.2, -0.2, 0.0]
    c["flags"] = [S.VALID, S.INCONSISTENT, S.VALID, S.EDGE_PEAK, S.VALID, S.OOB]
    # distances: 0, 0.78, 2.0, (edge peak: not a match), 2.0, (OOB: not a match)
    assert W.cmr(c, shift) == (2, 4)
    prior = np.array([[0, 0], [0, 0], [-2, 0], [0, 0], [0, -2], [0, 0]], np.int32)
    assert W.cmr(c, shift, prior) == (4, 4)


@pytest.mark.parametrize("v", [0.001, 0.01])
def test_gaussian_noise_statistics(v):
    img = np.full((400, 500), 0.5, np.float32)
    n = synth.gaussian_noise(img, v, 3) - img
    assert abs(n.mean()) < 4 * np.sqrt(v / n.size)
    assert abs(n.var() / v - 1) < 0.02
    np.testing.assert_array_equal(synth.gaussian_noise(img, v, 3), synth.gaussian_noise(img, v, 3))
    assert not np.array_equal(synth.gaussian_noise(img, v, 3), synth.gaussian_noise(img, v, 4))


@pytest.mark.parametrize("v", [0.01, 0.1])
def test_speckle_noise_statistics(v):
    rng = np.random.default_rng(0)
    img = rng.uniform(0.2, 1.0, (400, 500)).astype(np.float32)
    out = synth.speckle_noise(img, v, 5)
    rel = out.astype(np.float64) / img - 1.0
    assert abs(rel.mean()) < 4 * np.sqrt(v / rel.size)
    assert abs(rel.var() / v - 1) < 0.02
    h = np.sqrt(3 * v)
    assert rel.min() >= -h - 1e-5 and rel.max() <= h + 1e-5      # uniform on [-h, h]
    np.testing.assert_array_equal(synth.speckle_noise(np.zeros((8, 8), np.float32), v, 1), 0.0)


def test_sweep_levels_are_the_papers():
    assert synth.SWEEP["gaussian"] == [0.0, 0.001, 0.002, 0.003, 0.004, 0.005, 0.006, 0.007, 0.008, 0.009, 0.01]
    assert synth.SWEEP["speckle"] == [0.0, 0.01, 0.02, 0.03, 0.04, 0.05, 0.06, 0.07, 0.08, 0.09, 0.1]
    assert synth.SWEEP["m"] == 80
