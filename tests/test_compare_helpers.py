"""The GPU tests' comparison helpers, checked on constructed arrays (no GPU):
each kind of ambiguous pixel is accepted exactly inside its set of correct
results and rejected outside it."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import compare_ea, compare_mip


def test_mip_strict_pixels_use_relative_tolerance():
    ref = np.array([0.5, 40.0, -math.inf])
    compare_mip(np.array([0.5 + 0.9e-5, 40.0 + 39e-5, -math.inf]), ref, 1e-5)
    with pytest.raises(AssertionError):
        compare_mip(np.array([0.5 + 1.1e-5, 40.0, -math.inf]), ref, 1e-5)
    with pytest.raises(AssertionError):
        compare_mip(np.array([0.5, 40.0, 0.0]), ref, 1e-5)


def test_mip_nearest_ties_checked_against_bounds():
    ref = np.array([10.0, 10.0, 10.0, 0.0])
    fl = np.full(4, oracle.FLAG_HIT | oracle.FLAG_NEAREST_AMBIG, dtype=np.int32)
    bounds = np.array([[9.0, 11.0], [9.0, 11.0], [9.0, 11.0], [2.0, 3.5]])
    # the last pixel's maxima lie on both sides of the clip 3: 0 and [3, 3.5] are correct
    compare_mip(np.array([9.0, 11.0, 10.5, 0.0]), ref, 1e-5, fl, bounds, clip=3.0)
    compare_mip(np.array([9.0, 11.0, 10.5, 3.2]), ref, 1e-5, fl, bounds, clip=3.0)
    with pytest.raises(AssertionError):
        compare_mip(np.array([8.9, 11.0, 10.5, 0.0]), ref, 1e-5, fl, bounds, clip=3.0)
    with pytest.raises(AssertionError):
        compare_mip(np.array([9.0, 11.0, 10.5, 2.5]), ref, 1e-5, fl, bounds, clip=3.0)
    with pytest.raises(AssertionError):
        compare_mip(np.array([9.0, 11.0, 10.5, 0.0]), ref, 1e-5, fl, None, clip=3.0)


def test_mip_loose_kinds_checked_and_capped():
    n = 400
    ref = np.full(n, 5.0)
    fl = np.full(n, oracle.FLAG_HIT, dtype=np.int32)
    fl[0] |= oracle.FLAG_MIPCLIP_AMBIG
    fl[1] |= oracle.FLAG_GRAZE_AMBIG
    gpu = ref.copy()
    gpu[0] = 0.0          # floored at the clip: correct
    gpu[1] = -math.inf    # grazing ray missed: correct
    compare_mip(gpu, ref, 1e-5, fl)
    bad = gpu.copy()
    bad[0] = 4.0
    with pytest.raises(AssertionError):
        compare_mip(bad, ref, 1e-5, fl)
    # with a clip of 3: a maximum at the clip within the flag window is correct,
    # one outside it is not
    at = ref.copy()
    at[0] = 0.0
    gpu_c = at.copy()
    gpu_c[0] = 3.0 + 0.9e-4 * 3.0
    compare_mip(gpu_c, at, 1e-5, fl, clip=3.0)
    gpu_c[0] = 3.0 + 1.2e-4 * 3.0
    with pytest.raises(AssertionError):
        compare_mip(gpu_c, at, 1e-5, fl, clip=3.0)
    many = fl.copy()
    many[:10] |= oracle.FLAG_MIPCLIP_AMBIG  # 2.5 % of the pixels
    with pytest.raises(AssertionError):
        compare_mip(gpu, ref, 1e-5, many)


def test_ea_ambiguous_pixels_bounded_and_capped():
    n = 200
    ref = np.zeros((n, 4))
    ref[:, 3] = 0.5
    fl = np.full(n, oracle.FLAG_HIT, dtype=np.int32)
    fl[0] |= oracle.FLAG_ERT_AMBIG
    gpu = ref.copy()
    gpu[0, 3] += 0.009
    compare_ea(gpu, ref, 1e-5, fl)
    gpu[0, 3] += 0.002
    with pytest.raises(AssertionError):
        compare_ea(gpu, ref, 1e-5, fl)
