"""Seeded input generator: counter-based RNG, determinism, region regeneration, statistics."""
import math

import numpy as np
import pytest

import synth


def test_philox_known_answers():
    # Known-answer vectors published with the Philox4x32-10 definition
    # (Salmon et al., SC 2011; Random123 distribution).
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                               [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                             0x24126EA1]


def test_cube_deterministic_and_thread_independent():
    spec = synth.CubeSpec(37, 29, 23, seed=77, sources=synth.SourcePop(4, 5, 20, False, 2, 6, 2, 6))
    a = synth.cube(spec, threads=1)
    b = synth.cube(spec, threads=7)
    assert a.dtype == np.float32 and a.shape == (23, 29, 37)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    c = synth.cube(synth.CubeSpec(37, 29, 23, seed=78, sources=spec.sources))
    assert not np.array_equal(a, c)


def test_slab_regeneration_equals_full_cube():
    spec = synth.CubeSpec(40, 33, 50, seed=5, sources=synth.SourcePop(6, 3, 50, True, 1, 8, 2, 40))
    full = synth.cube(spec)
    for z0, nz in [(0, 1), (7, 13), (49, 1), (20, 30)]:
        part = synth.cube_slab(spec, z0, nz)
        assert np.array_equal(part, full[z0:z0 + nz])


def test_noise_statistics():
    spec = synth.CubeSpec(128, 128, 64, seed=11, sources=None)
    v = synth.cube(spec).astype(np.float64).ravel()
    n = v.size
    assert abs(v.mean()) < 5.0 / math.sqrt(n)
    assert abs(v.std() - 1.0) < 5.0 * math.sqrt(0.5 / n)
    # tail fraction above 3 sigma: P(Z>3) = 1.3499e-3
    p = (v > 3.0).mean()
    assert abs(p - 1.3499e-3) < 6 * math.sqrt(1.35e-3 / n)
    # Kolmogorov-Smirnov distance against the normal CDF
    from scipy import stats
    ks = stats.kstest(v[:200000], "norm")
    assert ks.pvalue > 1e-4


def test_sigma_scales_noise():
    a = synth.cube(synth.CubeSpec(16, 16, 16, seed=3, sigma=1.0))
    b = synth.cube(synth.CubeSpec(16, 16, 16, seed=3, sigma=4.0))
    assert np.array_equal(b, (a.astype(np.float64) * 4.0).astype(np.float32))


def test_source_catalogue_ranges():
    spec = synth.CubeSpec(512, 512, 1024, seed=1002,
                          sources=synth.SourcePop(200, 3.0, 50.0, True, 1.0, 8.0, 2.0, 40.0))
    s = synth.source_catalogue(spec)
    assert s.shape == (200, 6)
    assert (s[:, 0] >= 0).all() and (s[:, 0] <= 511).all()
    assert (s[:, 2] >= 0).all() and (s[:, 2] <= 1023).all()
    assert (s[:, 3] >= 3).all() and (s[:, 3] <= 50).all()
    assert (s[:, 4] >= 1).all() and (s[:, 4] <= 8).all()
    assert (s[:, 5] >= 2).all() and (s[:, 5] <= 40).all()
    # log-uniform amplitudes: log A roughly uniform -> median near sqrt(3*50)
    assert 6.0 < np.median(s[:, 3]) < 20.0


def test_single_source_profile():
    """Noise-free cube with one source equals the 3-D Gaussian at voxel centres."""
    spec = synth.CubeSpec(24, 20, 30, seed=9, noise=False,
                          sources=synth.SourcePop(1, 10, 10, False, 2, 2, 3, 3))
    src = synth.source_catalogue(spec)
    x0, y0, z0, A, ss, sz = src[0]
    v = synth.cube(spec)
    z, y, x = np.meshgrid(np.arange(30), np.arange(20), np.arange(24), indexing="ij")
    g = A * np.exp(-0.5 * (((x - x0) ** 2 + (y - y0) ** 2) / ss ** 2 + (z - z0) ** 2 / sz ** 2))
    inside = (np.abs(x - x0) <= 5 * ss) & (np.abs(y - y0) <= 5 * ss) & (np.abs(z - z0) <= 5 * sz)
    g = np.where(inside, g, 0.0)
    assert np.max(np.abs(v - g)) <= 1e-5 * A
    assert abs(float(v.max()) - A) < 0.2 * A  # centre lies between voxels


def test_workload_recipes():
    t = synth.tiny()
    assert (t.cube.nx, t.cube.ny, t.cube.nz) == (64, 64, 128)
    f = synth.full()
    assert (f.cube.nx, f.cube.ny, f.cube.nz) == (512, 512, 1024)
    assert (f.width, f.height) == (1024, 1024)
    cubes = synth.serving_cubes()
    assert len(cubes) == 8
    for c in cubes:
        assert 128 <= c.nx <= 1024 and 128 <= c.ny <= 1024 and 128 <= c.nz <= 512


def test_pixel_subset_distinct_and_in_range():
    px = synth.pixel_subset(4, 100, 37, 500)
    assert px.shape == (500, 2)
    assert (px[:, 0] >= 0).all() and (px[:, 0] < 100).all()
    assert (px[:, 1] >= 0).all() and (px[:, 1] < 37).all()
    assert len({(int(a), int(b)) for a, b in px}) == 500


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_axis_camera_is_axis_aligned(axis):
    cam = synth.axis_camera(64, 64, 128, axis, 256, 256)
    f = np.subtract(cam.target, cam.eye)
    assert np.count_nonzero(f) == 1
