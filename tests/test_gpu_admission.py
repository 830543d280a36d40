"""Serving under a device-memory budget: cubes registered with a host source
are admitted on demand and evicted while idle, least recently used first.

Checks that (1) with the budget at half of the registered cubes' bytes every
served request completes, cubes are uploaded and evicted along the way, and
each image is bit-identical to the same request rendered alone from a fully
resident cube; (2) single renders of registered cubes under the budget give
the same images; (3) a cube larger than the whole budget is refused; (4) the
serving workload's cubes (eight FP16 cubes of 128..1024 x 128..1024 x 128..512
voxels, images up to 2048^2), served under that budget, match the FP64
reference on sampled pixels of one response in ten: against the decoded codes
at the float32 tolerance and against the original values at the 16-bit one."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_16, TOL_F32, compare_ea, compare_mip, record, ref_render, wl_kwargs

pytestmark = pytest.mark.gpu


def need_bytes(info):
    """Device bytes the library admits a cube with: pool and per-cell statistics."""
    def a(b):
        return (b + 255) // 256 * 256
    slots = info.bricks_x * info.bricks_y * info.bricks_z
    return a(info.pool_bytes) + a(slots * 64 * 2 * 4)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def requests_for(r, specs, cubes, n, seed, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ci = int(rng.integers(0, len(specs)))
        sz = sizes[int(rng.integers(0, len(sizes)))]
        mode = "ea" if rng.random() < 0.5 else "mip"
        s = specs[ci]
        cam = synth.orbit_camera(s.nx, s.ny, s.nz, float(rng.uniform(0, 2 * math.pi)),
                                 float(rng.uniform(-math.pi / 4, math.pi / 4)))
        out.append((ci, sz, mode, cam))
    return out


def test_admission_under_half_budget():
    from paper_1001_2049_amd import Renderer, vr
    specs = [synth.CubeSpec(96, 80, 70, seed=77, sources=synth.SourcePop(6, 3, 50, True, 1, 8, 2, 20)),
             synth.CubeSpec(64, 64, 128, seed=1001, sources=synth.SourcePop(3, 5, 20, False, 2, 6, 2, 6)),
             synth.CubeSpec(100, 70, 60, seed=5, sources=synth.SourcePop(8, 3, 50, True, 1, 8, 2, 20)),
             synth.CubeSpec(70, 110, 90, seed=6, sources=synth.SourcePop(8, 3, 50, True, 1, 8, 2, 20))]
    vols = [synth.cube(s) for s in specs]
    storages = ["f32", "f32", "f16", "bf16"]
    tf = synth.ramp_tf(256, 1.0)
    ref_r = Renderer(0)
    r = None
    try:
        ref_cubes = [ref_r.upload(v, st) for v, st in zip(vols, storages)]
        ref_r.set_transfer_function(tf, 3.0, 20.0)
        ref_r.set_noise_clip(3.0, 1.0)
        needs = [need_bytes(ref_r.info(c)) for c in ref_cubes]
        budget = sum(needs) // 2
        assert budget >= max(needs)
        plan = requests_for(ref_r, specs, ref_cubes, 40, seed=21, sizes=[64, 100, 256, 300])
        alone = []
        for ci, sz, mode, cam in plan:
            ref_r.set_camera(cam)
            alone.append(to_np(ref_r.render(ref_cubes[ci], sz, sz, mode=mode)))

        print("admission: budget %d of %d bytes" % (budget, sum(needs)), flush=True)
        r = Renderer(0, budget_bytes=budget)
        cubes = [r.register(v, st) for v, st in zip(vols, storages)]
        assert all(r.info(c).resident == 0 and r.info(c).registered == 1 for c in cubes)
        r.set_transfer_function(tf, 3.0, 20.0)
        r.set_noise_clip(3.0, 1.0)
        # single renders under the budget (admission inside vr_render)
        for (ci, sz, mode, cam), want in list(zip(plan, alone))[:8]:
            r.set_camera(cam)
            got = to_np(r.render(cubes[ci], sz, sz, mode=mode))
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
            assert r.memory_stats()["used_bytes"] <= budget
        m0 = r.memory_stats()
        print("admission: single renders done", m0, flush=True)
        # served mix: all requests at once, two launches in flight
        outs = [r.output(sz, sz, mode) for _, sz, mode, _ in plan]
        for o in outs:
            o.fill_(math.nan)
        reqs = [r.request(cubes[ci], cam, sz, sz, o, mode=mode, clip=3.0)
                for (ci, sz, mode, cam), o in zip(plan, outs)]
        r.server_start(max_batch_requests=16, max_batch_tiles=64, max_inflight=2, use_graphs=1)
        try:
            tickets = [r.submit(q) for q in reqs]
            for k, t in enumerate(tickets):
                r.wait(t, timeout_s=120)
                print("admission: ticket %d done" % k, flush=True)
        finally:
            r.server_stop()
        for o, want in zip(outs, alone):
            got = to_np(o)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
        m1 = r.memory_stats()
        assert m1["used_bytes"] <= budget
        assert m1["uploads"] > m0["uploads"] and m1["evictions"] > 0, (m0, m1)
        assert m1["registered_cubes"] == 4 and m1["resident_cubes"] < 4
        # a cube that alone exceeds the budget is refused at registration
        big = np.zeros((200, 200, 200), np.float32)
        with pytest.raises(vr.VRError) as e:
            r.register(big, "f32")
        assert e.value.status == vr.VR_ENOMEM
    finally:
        if r is not None:
            r.close()
        ref_r.close()


def test_serving_workload_cubes_under_half_budget():
    """The serving workload's eight FP16 cubes, registered from host codes
    under half their total bytes; 40 requests (images 256^2..2048^2, EA and
    MIP) served together; every fourth response bit-identical to its alone
    render on a fully resident cube, and one in ten checked against the FP64
    reference on 400 sampled pixels."""
    import torch

    from paper_1001_2049_amd import Renderer
    specs = synth.serving_cubes(8)
    vols = [synth.cube(s, threads=16) for s in specs]
    codes = [oracle.to_f16_bits(v) for v in vols]
    tf = synth.ramp_tf(256, 1.0)
    plan = requests_for(None, specs, None, 40, seed=4243, sizes=[256, 512, 1024, 2048])
    r = ref_r = None
    try:
        ref_r = Renderer(0)
        ref_cubes = [ref_r.upload(c, "f16", src_dtype="f16") for c in codes]
        needs = [need_bytes(ref_r.info(c)) for c in ref_cubes]
        budget = max(sum(needs) // 2, max(needs))
        ref_r.set_transfer_function(tf, 3.0, 50.0)
        ref_r.set_noise_clip(3.0, 1.0)
        alone = {}
        for k, (ci, sz, mode, cam) in enumerate(plan):
            if k % 4 == 0:
                ref_r.set_camera(cam)
                alone[k] = to_np(ref_r.render(ref_cubes[ci], sz, sz, mode=mode))
        ref_r.close()
        ref_r = None
        torch.cuda.empty_cache()

        r = Renderer(0, budget_bytes=budget)
        cubes = [r.register(c, "f16", src_dtype="f16") for c in codes]
        r.set_transfer_function(tf, 3.0, 50.0)
        r.set_noise_clip(3.0, 1.0)
        outs = [r.output(sz, sz, mode) for _, sz, mode, _ in plan]
        reqs = [r.request(cubes[ci], cam, sz, sz, o, mode=mode, clip=3.0)
                for (ci, sz, mode, cam), o in zip(plan, outs)]
        r.server_start(max_batch_requests=64, max_batch_tiles=4096, max_inflight=2, use_graphs=1)
        try:
            tickets = [r.submit(q) for q in reqs]
            for t in tickets:
                r.wait(t, timeout_s=300)
        finally:
            r.server_stop()
        m = r.memory_stats()
        assert m["used_bytes"] <= budget and m["evictions"] > 0, m
        wl_base = dict(v0=3.0, v1=50.0, clip_k=3.0)
        for k, ((ci, sz, mode, cam), o) in enumerate(zip(plan, outs)):
            got_img = to_np(o)
            if k in alone:
                assert np.array_equal(got_img.view(np.uint32), alone[k].view(np.uint32)), k
            if k % 10 != 0:
                continue
            wl = synth.Workload("serve", specs[ci], sz, sz, **wl_base)
            kw = wl_kwargs(wl, tf)
            px = synth.pixel_subset(7000 + k, sz, sz, 400)
            got = got_img[px[:, 1], px[:, 0]]
            dec = ref_render(oracle.decode_bits(codes[ci], oracle.F16), kw, cam, sz, sz, mode,
                             "trilinear", pixels=px)
            orig = ref_render(vols[ci], kw, cam, sz, sz, mode, "trilinear", pixels=px,
                              amb_ert=TOL_16, amb_clip=TOL_16)
            if mode == "ea":
                a = compare_ea(got, dec["values"], TOL_F32, dec["flags"])
                g = compare_ea(got, orig["values"], TOL_16, orig["flags"], max_ambiguous_frac=0.05)
            else:
                a = compare_mip(got, dec["values"], TOL_F32, dec["flags"], dec.get("bounds"), clip=3.0)
                g = compare_mip(got, orig["values"], TOL_16, orig["flags"], orig.get("bounds"),
                                clip=3.0, amb_clip=TOL_16)
            record("served f16 %dx%dx%d %d %s arith" % (specs[ci].nx, specs[ci].ny, specs[ci].nz, sz, mode), a)
            record("served f16 %dx%dx%d %d %s gate" % (specs[ci].nx, specs[ci].ny, specs[ci].nz, sz, mode), g)
    finally:
        if r is not None:
            r.close()
        if ref_r is not None:
            ref_r.close()
