"""Cubes larger than the device-memory budget (the paper's data larger than a
GPU's memory, abstract and Sec. 2): a registered cube whose bricks do not fit
the budget is bricked into pinned host memory and rendered as sub-cubes of
brick layers, uploaded in turn, each to a partial image on the whole cube's
lattice, integrated front to back.

Checks that (1) with early termination off the streamed image matches the
FP64 reference's whole image and the renderer's fully resident image; (2)
with early termination on, where it acts within each sub-cube, it is at least
as opaque as the resident image and within the termination bound of it; (3)
sample counts add up to the whole lattice; (4) the device holds no more than
the budget."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, record, ref_render

pytestmark = pytest.mark.gpu


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("budget_mb", [24, 28])
def test_streamed_cube_matches_reference(budget_mb):
    from paper_1001_2049_amd import Renderer
    spec = synth.CubeSpec(160, 144, 200, seed=9090, sources=synth.SourcePop(10, 4, 40, True, 1.5, 6, 2, 20))
    vol = synth.cube(spec)
    tf = synth.ramp_tf(256, 1.0)
    cam = synth.orbit_camera(160, 144, 200, 0.8, 0.6)
    W, H = 240, 200
    budget = budget_mb << 20
    res_r = Renderer(0)
    r = Renderer(0, budget_bytes=budget)
    try:
        for x in (res_r, r):
            x.set_transfer_function(tf, 3.0, 40.0)
            x.set_noise_clip(3.0, 1.0)
            x.set_camera(cam)
        full = res_r.upload(vol, "f32")
        cube = r.register(vol, "f32")
        info = r.info(cube)
        assert info.pool_bytes > budget
        kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=40.0, clip=3.0, step=0.5)
        for mode in ("ea", "mip"):
            for ert in (2.0, 0.99):
                if mode == "mip" and ert < 1.0:
                    continue
                img, st = r.render(cube, W, H, mode=mode, ert=ert, stats=True)
                got = to_np(img)
                m = r.memory_stats()
                assert m["used_bytes"] <= budget, m
                resident, st_res = res_r.render(full, W, H, mode=mode, ert=ert, stats=True)
                resident = to_np(resident)
                assert st["samples_nominal"] == st_res["samples_nominal"]
                ert32 = float(np.float32(ert)) if ert < 1.0 else ert
                want = flags = ref = None
                if ert >= 1.0:
                    ref = ref_render(vol, dict(kw, ert=ert32), cam, W, H, mode, "trilinear")
                    want, flags = ref["image"], ref["flags"]
                if mode == "ea" and want is not None:
                    i1 = compare_ea(got, want, TOL_F32, flags)
                    assert np.max(np.abs(got - resident)) <= 2 * TOL_F32
                elif mode == "mip":
                    i1 = compare_mip(got, want, TOL_F32, flags, ref.get("bounds"), clip=3.0)
                    hit = np.isfinite(resident)
                    assert np.array_equal(hit, np.isfinite(got))
                else:
                    # with early termination: each sub-cube stops on its own, so the
                    # streamed image is at least as opaque and within the ERT bound
                    i1 = {"max_err_vs_resident": float(np.max(np.abs(got - resident)))}
                    assert np.all(got[..., 3] >= resident[..., 3] - 1e-5)
                    assert np.max(np.abs(got - resident)) <= 0.01 + TOL_F32
                record("streamed %s ert%s budget %dMB (%.1f ms vs resident %.1f ms)"
                       % (mode, ert, budget_mb, st["kernel_ms"], st_res["kernel_ms"]), i1)
    finally:
        r.close()
        res_r.close()


def test_streamed_frames_reuse_sub_cubes_and_yield_them():
    """Consecutive frames walk the sub-cubes in opposite orders, starting on the
    two the frame before left in device memory: the images stay identical bit
    for bit, and those buffers give way to an upload that needs the room."""
    from paper_1001_2049_amd import Renderer
    spec = synth.CubeSpec(160, 144, 200, seed=9091, sources=synth.SourcePop(10, 4, 40, True, 1.5, 6, 2, 20))
    vol = synth.cube(spec)
    W, H = 200, 176
    budget = 24 << 20
    r = Renderer(0, budget_bytes=budget)
    try:
        r.set_transfer_function(synth.ramp_tf(256, 1.0), 3.0, 40.0)
        r.set_noise_clip(3.0, 1.0)
        r.set_camera(synth.orbit_camera(160, 144, 200, 2.3, -0.4))
        cube = r.register(vol, "f32")
        assert r.info(cube).pool_bytes > budget
        frames = [to_np(r.render(cube, W, H, mode=m, ert=2.0)) for m in ("ea", "ea", "ea", "mip", "mip")]
        for a, b in [(0, 1), (1, 2), (3, 4)]:
            assert np.array_equal(frames[a].view(np.uint32), frames[b].view(np.uint32)), (a, b)
        held = r.memory_stats()["used_bytes"]
        # an uploaded cube that fits only once the kept buffers are freed
        small = synth.cube(synth.CubeSpec(128, 128, 128, seed=9092, sources=synth.SourcePop(2, 4, 20, True, 2, 4, 2, 6)))
        assert budget - held < 4 * 128 ** 3  # less than its voxels' bytes, let alone its bricks'
        other = r.upload(small, "f32")
        assert r.memory_stats()["used_bytes"] <= budget
        assert r.memory_stats()["used_bytes"] - r.info(other).pool_bytes < held
        r.release(other)
        again = to_np(r.render(cube, W, H, mode="ea", ert=2.0))
        assert np.array_equal(again.view(np.uint32), frames[0].view(np.uint32))
    finally:
        r.close()


def test_progressive_levels_of_a_streamed_cube():
    """A cube larger than the budget gets resident coarse levels, built from its
    pinned bricks: levels 3, 2, 1 are the method on the level-L cube (FP64
    reference), and level 0 is the streamed full render, bit for bit."""
    from oracle import levels
    from paper_1001_2049_amd import Renderer
    spec = synth.CubeSpec(160, 144, 200, seed=9093, sources=synth.SourcePop(10, 4, 40, True, 1.5, 6, 2, 20))
    vol = synth.cube(spec)
    tf = synth.ramp_tf(256, 1.0)
    cam = synth.orbit_camera(160, 144, 200, 1.3, 0.45)
    W, H = 180, 150
    budget = 28 << 20
    r = Renderer(0, budget_bytes=budget)
    try:
        r.set_transfer_function(tf, 3.0, 40.0)
        r.set_noise_clip(3.0, 1.0)
        r.set_camera(cam)
        cube = r.register(vol, "f32")
        assert r.info(cube).pool_bytes > budget
        out = r.output(W, H, "ea")
        kw = dict(v0=3.0, v1=40.0, clip=3.0, step=0.5, ert=float(np.float32(0.99)))
        seen = []
        for _ in range(5):
            info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
            if info["converged"]:
                break
            assert r.memory_stats()["used_bytes"] <= budget
            L = info["level"]
            seen.append(L)
            got = to_np(out)
            if L > 0:
                assert info["level_cube"] == 1, info
                wl, hl = levels.level_size(W, H, L)
                low = got[::2 ** L, ::2 ** L]
                ref = ref_render(levels.level_volume(vol, L), dict(kw, tf=levels.level_tf(tf, L)),
                                 levels.level_camera(cam, L), wl, hl, "ea", "trilinear")
                record("streamed progressive level %d" % L, compare_ea(low, ref["image"], TOL_F32, ref["flags"]))
            else:
                full = to_np(r.render(cube, W, H, mode="ea"))
                assert np.array_equal(got.view(np.uint32), full.view(np.uint32))
        assert seen == [3, 2, 1, 0], seen
    finally:
        r.close()
