"""Progressive (coarse-to-fine) rendering for the thin client's interactive
loop (paper Fig. 1 caption; Sec. 3.1, process step 4).

Checks that (1) each coarse level is the method applied to the cube's level-L
resolution pyramid (2x2x2 block means, the camera carried into level
coordinates, extinction scaled by 2^L: ``oracle.levels``), rendered at the
reduced size and enlarged by pixel replication, within the float32 tolerance
of the FP64 reference; (2) repeated calls on one view refine level by level
down to the full image, which is exactly vr_render's, and then report
convergence; (3) a new view restarts at a coarse level chosen from the
measured cost and the budget; (4) where a level cube cannot be used (an axis
below two voxels, no room in the memory budget) the level is the full cube
rendered with a lattice step 2^L times longer, bit for bit, and the level
cubes are the first memory to go when an upload needs room."""
import math

import numpy as np
import pytest

import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, ref_render
from oracle import levels

pytestmark = pytest.mark.gpu


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def enlarge(low, W, H, L):
    ys = np.minimum(np.arange(H) >> L, low.shape[0] - 1)
    xs = np.minimum(np.arange(W) >> L, low.shape[1] - 1)
    return low[ys][:, xs]


@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_levels_refine_to_the_full_image(mode):
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    try:
        spec = synth.CubeSpec(80, 72, 96, seed=808, sources=synth.SourcePop(6, 4, 30, True, 1.5, 5, 2, 12))
        vol = synth.cube(spec)
        cube = r.upload(vol, "f32")
        tf = synth.ramp_tf(256, 1.0)
        r.set_transfer_function(tf, 3.0, 30.0)
        r.set_noise_clip(3.0, 1.0)
        cam = synth.orbit_camera(80, 72, 96, 0.9, 0.4)
        r.set_camera(cam)
        W, H = 203, 150
        out = r.output(W, H, mode)
        seen, imgs, infos = [], [], []
        for _ in range(6):
            info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode=mode)
            if info["converged"]:
                break
            seen.append(info["level"])
            infos.append(info)
            imgs.append(to_np(out).copy())
        assert seen == [3, 2, 1, 0], seen
        assert all(i["level_cube"] == 1 for i in infos[:3]), infos
        full = to_np(r.render(cube, W, H, mode=mode))
        assert np.array_equal(imgs[-1].view(np.uint32), full.view(np.uint32))
        # each coarse level: the method on the level-L cube, enlarged
        kw = dict(v0=3.0, v1=30.0, clip=3.0, step=0.5, ert=float(np.float32(0.99)))
        for k, L in enumerate([3, 2, 1]):
            wl, hl = levels.level_size(W, H, L)
            low = imgs[k][::2 ** L, ::2 ** L]
            assert low.shape[:2] == (hl, wl)
            assert np.array_equal(imgs[k].view(np.uint32), enlarge(low, W, H, L).view(np.uint32))
            ref = ref_render(levels.level_volume(vol, L), dict(kw, tf=levels.level_tf(tf, L)),
                             levels.level_camera(cam, L), wl, hl, mode, "trilinear")
            if mode == "ea":
                compare_ea(low, ref["image"], TOL_F32, ref["flags"])
            else:
                compare_mip(low, ref["image"], TOL_F32, ref["flags"], ref.get("bounds"), clip=3.0)
            # about 8^L times fewer samples than the full image
            assert infos[k]["samples_nominal"] * 8 ** L < 1.3 * infos[3]["samples_nominal"]
        # a new view restarts coarse; a generous budget gives the full level at once
        r.set_camera(synth.orbit_camera(80, 72, 96, 2.0, -0.3))
        info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode=mode)
        assert info["level"] == 3 and info["predicted_ms"] > 0
        r.set_camera(synth.orbit_camera(80, 72, 96, 2.5, -0.3))
        info = r.render_progressive(cube, W, H, out, budget_ms=1e3, max_level=3, mode=mode)
        assert info["level"] == 0
        info = r.render_progressive(cube, W, H, out, budget_ms=1e3, max_level=3, mode=mode)
        assert info["converged"] == 1
    finally:
        r.close()


def _long_step_level(r, cube, W, H, L, mode):
    """The fallback definition of level L: the full cube at ceil(W/2^L) x
    ceil(H/2^L) with a lattice step 2^L times longer, enlarged."""
    wl, hl = levels.level_size(W, H, L)
    return enlarge(to_np(r.render(cube, wl, hl, mode=mode, step=0.5 * 2 ** L)), W, H, L)


def test_level_with_a_short_axis_uses_the_full_cube():
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    try:
        # nz = 7: levels 1 and 2 have 4 and 2 planes, level 3 would have 1
        spec = synth.CubeSpec(48, 40, 7, seed=812, sources=synth.SourcePop(3, 4, 30, True, 1.5, 4, 1, 3))
        vol = synth.cube(spec)
        cube = r.upload(vol, "f32")
        r.set_transfer_function(synth.ramp_tf(256, 1.0), 3.0, 30.0)
        r.set_noise_clip(3.0, 1.0)
        r.set_camera(synth.orbit_camera(48, 40, 7, 0.7, 0.5))
        W, H = 96, 72
        out = r.output(W, H, "ea")
        info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        assert info["level"] == 3 and info["level_cube"] == 0
        got = to_np(out).copy()
        assert np.array_equal(got.view(np.uint32), _long_step_level(r, cube, W, H, 3, "ea").view(np.uint32))
        info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        assert info["level"] == 2 and info["level_cube"] == 1
    finally:
        r.close()


def test_level_cubes_yield_to_uploads_under_a_budget():
    from paper_1001_2049_amd import Renderer
    spec = synth.CubeSpec(96, 80, 112, seed=813, sources=synth.SourcePop(6, 4, 30, True, 1.5, 5, 2, 12))
    vol = synth.cube(spec)
    cam = synth.orbit_camera(96, 80, 112, 1.1, 0.3)
    W, H = 128, 112

    def setup(r):
        r.set_transfer_function(synth.ramp_tf(256, 1.0), 3.0, 30.0)
        r.set_noise_clip(3.0, 1.0)
        r.set_camera(cam)

    # sizes: one cube, and its three coarse levels
    r = Renderer(0)
    try:
        setup(r)
        a = r.upload(vol, "f32")
        u_cube = r.memory_stats()["used_bytes"]
        out = r.output(W, H, "ea")
        r.render_progressive(a, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        u_levels = r.memory_stats()["used_bytes"] - u_cube
        assert u_levels > 0
    finally:
        r.close()
    # room for two cubes and half the levels: the levels fit beside one cube
    r = Renderer(0, budget_bytes=2 * u_cube + u_levels // 2)
    try:
        setup(r)
        a = r.upload(vol, "f32")
        out = r.output(W, H, "ea")
        info = r.render_progressive(a, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        assert info["level"] == 3 and info["level_cube"] == 1
        assert r.memory_stats()["used_bytes"] == u_cube + u_levels
        b = r.upload(vol, "f32")  # fits once the levels are gone
        assert r.memory_stats()["used_bytes"] == 2 * u_cube
        r.set_camera(synth.orbit_camera(96, 80, 112, 2.1, -0.2))
        info = r.render_progressive(a, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        assert info["level"] == 3 and info["level_cube"] == 0
        got = to_np(out).copy()
        assert np.array_equal(got.view(np.uint32), _long_step_level(r, a, W, H, 3, "ea").view(np.uint32))
        assert b != a
    finally:
        r.close()
