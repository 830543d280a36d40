"""Progressive (coarse-to-fine) rendering for the thin client's interactive
loop (paper Fig. 1 caption; Sec. 3.1, process step 4).

Checks that (1) a coarse level is exactly the renderer's image at the
reduced size and longer step, enlarged by pixel replication, and that image
matches the FP64 reference rendered at that size and step; (2) repeated calls
on one view refine level by level down to the full image, which is exactly
vr_render's, and then report convergence; (3) a new view restarts at a coarse
level chosen from the measured cost and the budget: a tiny budget gives the
coarsest level, a generous one the full level."""
import math

import numpy as np
import pytest

import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, ref_render

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
        levels, imgs = [], []
        for _ in range(6):
            info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode=mode)
            if info["converged"]:
                break
            levels.append(info["level"])
            imgs.append(to_np(out).copy())
        assert levels == [3, 2, 1, 0], levels
        full = to_np(r.render(cube, W, H, mode=mode))
        assert np.array_equal(imgs[-1].view(np.uint32), full.view(np.uint32))
        # level 2 = the renderer at a quarter of the size and 4x the step, enlarged
        L = 2
        wl, hl = (W + 3) >> L, (H + 3) >> L
        low = to_np(r.render(cube, wl, hl, mode=mode, step=0.5 * 4))
        assert np.array_equal(imgs[1].view(np.uint32), enlarge(low, W, H, L).view(np.uint32))
        # ... and that reduced image is the method at that lattice
        kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=30.0, clip=3.0, step=2.0,
                  ert=float(np.float32(0.99)))
        ref = ref_render(vol, kw, cam, wl, hl, mode, "trilinear")
        if mode == "ea":
            compare_ea(low, ref["image"], TOL_F32, ref["flags"])
        else:
            compare_mip(low, ref["image"], TOL_F32, ref["flags"], ref.get("bounds"), clip=3.0)
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
