"""Pins of the per-channel noise reference (oracle/noise.py): the robust noise
estimate of each frequency channel and rendering in units of it (the paper's
attention to data of low signal-to-noise ratio, abstract and Sec. 2)."""
import math
import statistics

import numpy as np

import oracle
import synth
from oracle import noise


def test_worked_example_by_hand():
    # values 3 1 4 1 5 9 2 6: sorted 1 1 2 3 4 5 6 9, lower median (index 3) = 3;
    # |v - 3| = 0 2 1 2 2 6 1 3, sorted 0 1 1 2 2 2 3 6, lower median = 2
    ch = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float32).reshape(1, 2, 4)
    med, mad, sig = noise.channel_stats(ch)
    assert med[0] == 3.0 and mad[0] == 2.0
    assert sig[0] == 1.4826 * 2.0
    # odd count: 7 values, median index 3
    ch = np.array([10, -2, 7, 0, 3, 3, 100], np.float32).reshape(1, 1, 7)
    med, mad, _ = noise.channel_stats(ch)
    assert med[0] == 3.0 and mad[0] == 4.0  # |v-3| = 7 5 4 3 0 0 97 -> 0 0 3 [4] 5 7 97


def test_matches_standard_library_lower_median():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 10, 11, 257):
        x = rng.standard_normal(n).astype(np.float32)
        ch = x.reshape(1, 1, n)
        med, mad, _ = noise.channel_stats(ch)
        m = statistics.median_low([float(v) for v in x])
        assert med[0] == m
        assert mad[0] == statistics.median_low([abs(float(v) - m) for v in x])


def test_shift_and_power_of_two_scale():
    rng = np.random.default_rng(4)
    x = rng.integers(-1000, 1000, size=(3, 16, 16)).astype(np.float32)
    med, mad, sig = noise.channel_stats(x)
    med2, mad2, sig2 = noise.channel_stats(x + np.float32(37.0))
    assert np.array_equal(med2, med + 37.0) and np.array_equal(mad2, mad)
    med4, mad4, _ = noise.channel_stats(x * np.float32(4.0))
    assert np.array_equal(med4, 4 * med) and np.array_equal(mad4, 4 * mad)


def test_recovers_known_gaussian_noise_profile():
    """Pure noise with a per-channel level: the estimate follows the profile
    within a few standard errors (MAD estimator, n = 96*96 per channel)."""
    spec = synth.CubeSpec(96, 96, 64, seed=31, sources=None)
    prof = synth.band_noise_profile(64)
    vol = synth.cube_profiled(spec, prof)
    _, _, sig = noise.channel_stats(vol)
    rel = sig / prof - 1.0
    se = 1.1 / math.sqrt(96 * 96)  # relative standard error of the MAD estimate, ~1.1/sqrt(n)
    assert np.max(np.abs(rel)) < 5 * se, np.max(np.abs(rel))
    assert abs(np.mean(rel)) < 3 * se / math.sqrt(64) + 2e-3


def test_robust_to_bright_sources():
    """Sources occupying a few per cent of a channel leave the estimate near
    the noise level, while the plain standard deviation is inflated."""
    spec = synth.CubeSpec(64, 64, 32, seed=9,
                          sources=synth.SourcePop(3, 20.0, 50.0, False, 1.0, 1.5, 30.0, 40.0))
    vol = synth.cube(spec)
    _, _, sig = noise.channel_stats(vol)
    std = vol.reshape(32, -1).std(axis=1)
    assert np.all(np.abs(sig - 1.0) < 0.08), sig
    assert np.max(std) > 1.5


def test_scaled_render_equals_global_clip_for_flat_profile():
    """With the same noise level s in every channel, rendering the scaled cube
    with clip k and a transfer function over [a, b] equals rendering the raw
    cube with clip k*s over [a*s, b*s] (float64, up to rounding)."""
    spec = synth.CubeSpec(40, 36, 30, seed=12, sources=synth.SourcePop(4, 5, 20, False, 2, 5, 2, 6))
    s = 2.5
    vol = (synth.cube(spec).astype(np.float64) * s)
    div = np.full(30, s)
    scaled = noise.scaled_cube(vol, div)
    tf = synth.ramp_tf(64, 1.0).astype(np.float64)
    cam = synth.orbit_camera(40, 36, 30, 0.7, 0.3)
    common = dict(tf=tf, step=0.5, ert=2.0, camera=cam, width=48, height=40)
    a = oracle.render(scaled, mode=oracle.EA, v0=3.0, v1=20.0, clip=3.0, **common)
    b = oracle.render(vol, mode=oracle.EA, v0=3.0 * s, v1=20.0 * s, clip=3.0 * s, **common)
    assert np.max(np.abs(a["image"] - b["image"])) < 1e-12
    am = oracle.render(scaled, mode=oracle.MIP, clip=3.0, **common)
    bm = oracle.render(vol, mode=oracle.MIP, clip=3.0 * s, **common)
    hit = np.isfinite(bm["image"])
    assert np.array_equal(hit, np.isfinite(am["image"]))
    assert np.max(np.abs(am["image"][hit] * s - bm["image"][hit])) < 1e-9
