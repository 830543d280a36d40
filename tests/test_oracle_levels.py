"""Pins of the reference's coarse levels (the progressive loop's resolution
pyramid) against invariants and closed forms, never against themselves:

* averaging is exact on constant and on linear fields, where the level-L
  voxel takes the field's value at its centre 2^L X + (2^L - 1)/2 (this fixes
  the axis order, the pairing of indices and the centre offset);
* 2 x 2 x 2 block means preserve the total over even-sized cubes;
* a cube whose voxels are each repeated twice along every axis averages back
  to itself, also when the last copy of an axis is cut off (odd sizes: the
  edge clamp);
* rendering a uniform medium at level L with the carried camera and the
  scaled extinction gives the opacity 1 - exp(-kappa L_fine) of the
  full-resolution chord along the same pixel's ray (this fixes the camera
  mapping, perspective and orthographic, and the extinction scale).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import levels
from test_oracle_pins import basis, face_clip_chord, ramp64, random_poses, window_positions


def test_constant_cube_stays_constant_at_every_level():
    for shape in [(8, 12, 16), (7, 5, 9), (3, 2, 5)]:
        vol = np.full(shape, 4.25)
        for L in range(4):
            lv = levels.level_volume(vol, L)
            assert lv.shape == levels.level_shape(shape, L)
            assert np.all(lv == 4.25)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_linear_field_takes_its_value_at_the_coarse_voxel_centre(L):
    nz, ny, nx = 16, 24, 40
    a, bx, by, bz = 0.7, 0.013, -0.029, 0.041

    def field(x, y, z):
        return a + bx * x + by * y + bz * z

    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lv = levels.level_volume(field(x, y, z), L)
    k = 2 ** L
    Z, Y, X = np.meshgrid(*[np.arange(n) for n in lv.shape], indexing="ij")
    off = (k - 1) / 2.0
    want = field(k * X + off, k * Y + off, k * Z + off)
    assert np.max(np.abs(lv - want)) < 1e-12


def test_block_means_preserve_the_total_on_even_cubes():
    rng = np.random.default_rng(7)
    vol = rng.normal(size=(16, 8, 24))
    for L in (1, 2, 3):
        assert abs(levels.level_volume(vol, L).sum() * 8 ** L - vol.sum()) < 1e-9


@pytest.mark.parametrize("cut", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_doubled_voxels_average_back_including_odd_edges(cut):
    rng = np.random.default_rng(11)
    v = rng.normal(size=(5, 6, 7))
    big = np.repeat(np.repeat(np.repeat(v, 2, axis=0), 2, axis=1), 2, axis=2)
    big = big[:big.shape[0] - cut[0], :big.shape[1] - cut[1], :big.shape[2] - cut[2]]
    # equal up to the rounding of the 8-term sum (a wrong pairing errs by O(1))
    assert np.max(np.abs(levels.downsample(big) - v)) <= 1e-15 * np.max(np.abs(v))


def _pinhole_ray(cam, W, H, i, j):
    """Pixel (i, j)'s ray from the camera definition (pinhole: the image plane
    at unit distance spans tan(fovy / 2) vertically, row 0 at the top)."""
    f, r, u = basis(cam)
    h = math.tan(math.radians(cam.fovy_deg) / 2.0)
    a = W / H
    d = f + (2.0 * (i + 0.5) / W - 1.0) * h * a * r + (1.0 - 2.0 * (j + 0.5) / H) * h * u
    return np.asarray(cam.eye, dtype=np.float64), d / np.linalg.norm(d)


@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("pose", range(3))
def test_uniform_medium_keeps_its_opacity_at_coarse_levels(L, pose):
    N = (16, 20, 24)  # x, y, z: even at both levels
    v = 7.3
    vol = np.full(N[::-1], v)
    v0, v1, kmax = 2.0, 12.0, 0.8
    tf = ramp64(256, kmax)
    kappa = kmax * (v - v0) / (v1 - v0)
    cam = random_poses(300 + pose, N, 3)[pose]
    W, H = 21, 15
    res = oracle.render(levels.level_volume(vol, L), mode=oracle.EA, tf=levels.level_tf(tf, L),
                        v0=v0, v1=v1, camera=levels.level_camera(cam, L), width=W, height=H,
                        step=0.5, ert=2.0)
    img = res["image"]
    nhit = 0
    for j in range(H):
        for i in range(W):
            o, d = _pinhole_ray(cam, W, H, i, j)
            ch = face_clip_chord(o, d, N, False)
            if ch is None:
                assert np.max(np.abs(img[j, i])) < 1e-9
                continue
            nhit += 1
            assert abs(img[j, i, 3] - (1.0 - math.exp(-kappa * (ch[1] - ch[0])))) < 1e-12
    assert nhit > 20


@pytest.mark.parametrize("L", [1, 2])
def test_orthographic_window_shrinks_with_the_level(L):
    N = (16, 20, 24)
    v = 9.0
    vol = np.full(N[::-1], v)
    v0, v1, kmax = 2.0, 12.0, 0.5
    tf = ramp64(256, kmax)
    kappa = kmax * (v - v0) / (v1 - v0)
    c = (np.asarray(N) - 1) / 2.0
    cam = synth.Camera(eye=tuple(c + np.array([40.0, 25.0, 31.0])), target=tuple(c + 0.3),
                       up=(0.0, 0.0, 1.0), ortho=True, ortho_w=34.0, ortho_h=26.0)
    W, H = 17, 13
    res = oracle.render(levels.level_volume(vol, L), mode=oracle.EA, tf=levels.level_tf(tf, L),
                        v0=v0, v1=v1, camera=levels.level_camera(cam, L), width=W, height=H,
                        step=0.5, ert=2.0)
    f, r, u = basis(cam)
    sx, sy = window_positions(cam, W, H)
    nhit = 0
    for j in range(H):
        for i in range(W):
            o = np.asarray(cam.target) + sx[i] * r + sy[j] * u
            ch = face_clip_chord(o, f, N, True)
            if ch is None:
                continue
            nhit += 1
            assert abs(res["image"][j, i, 3] - (1.0 - math.exp(-kappa * (ch[1] - ch[0])))) < 1e-12
    assert nhit > 20
