"""The large workload: a 2048 x 2048 x 4096 cube (noise plus 5000 sources)
stored as FP16, a 2048 x 2048 perspective view with the transfer function
clipped at 4 sigma (most cells are empty and skipped), and a 64-view orbit
rendered in one batched launch.

The cube is generated on the GPU with the seeded generator (synth), rounded
to FP16 codes (round to nearest even) and copied to the host for the
reference, which reads exactly those codes; the renderer uploads the same
float32 values and rounds them itself.  Sampled pixels are compared with the
FP64 reference at the float32 tolerance (arithmetic check on decoded values),
and batch members with their single renders bit for bit."""
import math
import os
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, record, ref_render, wl_kwargs

pytestmark = pytest.mark.gpu


def orbit64(spec, i, W):
    return synth.orbit_camera(spec.nx, spec.ny, spec.nz, 2.0 * math.pi * i / 64, math.radians(20.0))


@pytest.fixture(scope="module")
def large():
    import torch
    from paper_1001_2049_amd import Renderer
    synth.gpu_lib()  # built by __graft_entry__.build()
    wl = synth.large()
    spec = wl.cube
    vals = torch.empty((spec.nz, spec.ny, spec.nx), dtype=torch.float32, device="cuda")
    synth.cube_gpu(spec, vals)
    r = Renderer(0)
    cube = r.upload(vals, "f16")
    # compulsory bytes of a view that sees the whole cube: the FP16 voxels of
    # the 8^3 cells holding a value at or above the clip (no other cell can
    # contribute), counted on the float32 values, 256 planes at a time
    active_cells = 0
    with torch.no_grad():
        for z0 in range(0, spec.nz, 256):
            cm = torch.nn.functional.max_pool3d(vals[z0:z0 + 256].reshape(1, 1, -1, spec.ny, spec.nx), 8)
            active_cells += int((cm >= wl.clip_k * spec.sigma).sum().item())
            del cm
    codes = np.empty((spec.nz, spec.ny, spec.nx), dtype=np.uint16)
    for z0 in range(0, spec.nz, 256):
        codes[z0:z0 + 256] = vals[z0:z0 + 256].half().cpu().numpy().view(np.uint16)
    del vals
    torch.cuda.empty_cache()
    tf = synth.ramp_tf(256, wl.kappa_max)
    r.set_transfer_function(tf, wl.v0, wl.v1)
    r.set_noise_clip(wl.clip_k, 1.0)
    yield wl, r, cube, codes, tf, active_cells
    r.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_large_cube_sampled_pixels(large, mode):
    import torch
    wl, r, cube, codes, tf, active_cells = large
    W = H = wl.width
    cam = orbit64(wl.cube, 0, W)
    r.set_camera(cam)
    img, st = r.render(cube, W, H, mode=mode, stats=True)
    torch.cuda.synchronize()
    got_img = img.cpu().numpy()
    px = synth.pixel_subset(777, W, H, 16384)  # a seeded 16384-pixel subset
    got = got_img[px[:, 1], px[:, 0]]
    t0 = time.perf_counter()
    ref = ref_render(codes, wl_kwargs(wl, tf), cam, W, H, mode, "trilinear", pixels=px,
                     vox_dtype=oracle.F16, threads=os.cpu_count())
    t_ref = time.perf_counter() - t0
    # the reference on the sampled pixels only: per ray, and extrapolated to
    # the whole frame (an extrapolation, stated as such)
    print("large %s: reference %.4f ms per ray on %d threads (%d rays), full frame "
          "extrapolated %.0f s" % (mode, t_ref * 1e3 / len(px), os.cpu_count(), len(px),
                                   t_ref / len(px) * W * H), flush=True)
    if mode == "ea":
        info = compare_ea(got, ref["values"], TOL_F32, ref["flags"])
    else:
        info = compare_mip(got, ref["values"], TOL_F32, ref["flags"], ref.get("bounds"),
                           clip=wl.clip_k * wl.cube.sigma)
    record("large f16 2048 %s sampled" % mode, info)
    print("large %s stats=%s" % (mode, st))
    ncells = (wl.cube.nx // 8) * (wl.cube.ny // 8) * (wl.cube.nz // 8)
    compulsory = active_cells * 512 * 2 + W * H * (16 if mode == "ea" else 4)
    print("large %s: %d of %d cells active (%.1f %%), compulsory %.2f GB, %.0f GB/s = %.3f of 8 TB/s"
          % (mode, active_cells, ncells, 100.0 * active_cells / ncells, compulsory / 1e9,
             compulsory / (st["kernel_ms"] * 1e-3) / 1e9, compulsory / (st["kernel_ms"] * 1e-3) / 8e12))
    assert st["cells_skipped"] > 0 and st["samples_exec"] < st["samples_nominal"]


def test_large_orbit_batch_equals_single(large):
    """The 64-view orbit in one persistent launch and as 64 single launches on
    the same views: every view bit-identical, both timed with HIP events."""
    import torch
    wl, r, cube, codes, tf, _ = large
    W = H = wl.width
    outs = [r.output(W, H, "ea") for _ in range(64)]
    reqs = [r.request(cube, orbit64(wl.cube, i, W), W, H, outs[i], mode="ea", clip=wl.clip_k)
            for i in range(64)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r.render_batch(reqs)
    e1.record()
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1)
    single = r.output(W, H, "ea")
    single_ms = []
    for i in range(64):
        r.set_camera(orbit64(wl.cube, i, W))
        e0.record()
        r.render(cube, W, H, mode="ea", out=single)
        e1.record()
        torch.cuda.synchronize()
        single_ms.append(e0.elapsed_time(e1))
        assert torch.equal(single.view(torch.int32), outs[i].view(torch.int32)), i
    print("large orbit: one batched launch %.1f ms (%.2f ms per view); 64 single launches %.1f ms "
          "(%.2f ms per view, min %.2f, max %.2f)" % (batch_ms, batch_ms / 64, sum(single_ms),
                                                      sum(single_ms) / 64, min(single_ms), max(single_ms)))


def test_large_cube_streamed_under_a_budget(large):
    """The same cube registered from host memory (its FP16 codes) under a 16 GiB
    budget, about a third of its bricks: bricked into pinned host memory and
    streamed over PCIe in sub-cubes of brick layers.  With early termination
    off (where sub-cube partials compose to the whole image up to rounding) the
    frame matches the resident render; both frames' wall-clock times are
    reported."""
    import torch
    from paper_1001_2049_amd import Renderer
    wl, r, cube, codes, tf, _ = large
    W = H = wl.width
    cam = orbit64(wl.cube, 0, W)
    r.set_camera(cam)
    kw = dict(mode="ea", ert=2.0)
    resident = r.render(cube, W, H, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.render(cube, W, H, out=resident, **kw)
    torch.cuda.synchronize()
    res_ms = 1e3 * (time.perf_counter() - t0)
    budget = 16 << 30
    rs = Renderer(0, budget_bytes=budget)
    try:
        rs.set_transfer_function(tf, wl.v0, wl.v1)
        rs.set_noise_clip(wl.clip_k, 1.0)
        rs.set_camera(cam)
        sc = rs.register(codes, "f16", src_dtype="f16")
        assert rs.info(sc).pool_bytes > budget
        out = rs.output(W, H, "ea")
        times = []
        for _ in range(2):  # the first frame also bricks the cube into pinned host memory
            t0 = time.perf_counter()
            rs.render(sc, W, H, out=out, **kw)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        assert rs.memory_stats()["used_bytes"] <= budget
        diff = float((out - resident).abs().max().item())
        record("large streamed ea", {"max_abs_diff_vs_resident": diff, "first_frame_ms": times[0],
                                     "frame_ms": times[1], "resident_ms": res_ms,
                                     "pool_bytes": int(rs.info(sc).pool_bytes), "budget": budget})
        assert diff <= TOL_F32, diff
    finally:
        rs.close()
        torch.cuda.empty_cache()


def test_large_cube_progressive_levels(large):
    """The progressive loop on the resident 32 GiB cube: the first call builds
    its coarse levels (2x2x2 block means on the device) and shows level 3;
    each further call refines, and level 0 is the full render bit for bit.
    Level and build times are reported."""
    import torch
    wl, r, cube, codes, tf, _ = large
    W = H = wl.width
    r.set_camera(orbit64(wl.cube, 5, W))
    out = r.output(W, H, "ea")
    seen = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = r.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=3, mode="ea")
        torch.cuda.synchronize()
        wall = 1e3 * (time.perf_counter() - t0)
        if info["converged"]:
            break
        seen.append(info["level"])
        print("large progressive level %d: %.2f ms on the device, %.1f ms for the call, level cube %d"
              % (info["level"], info["ms"], wall, info["level_cube"]), flush=True)
        if info["level"] > 0:
            assert info["level_cube"] == 1
    assert seen == [3, 2, 1, 0], seen
    full = r.render(cube, W, H, mode="ea")
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), full.view(torch.int32))
