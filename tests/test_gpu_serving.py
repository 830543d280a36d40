"""Serving form on the GPU: continuous batching through vr_submit / vr_wait.

Checks that (1) each request's image is bit-identical when served alone and
when served in a mix of concurrent requests of different sizes, modes and
cubes; (2) graph-replayed launches give the same images as direct launches
over several replays with eager work in between; (3) served images match the
single-image renderer and, on sampled pixels, the FP64 reference; (4) state
errors are reported (submit without a server, releasing a cube with queued
requests)."""
import math
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, ref_render, wl_kwargs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    specs = [synth.CubeSpec(64, 64, 128, seed=1001, sources=synth.SourcePop(3, 5, 20, False, 2, 6, 2, 6)),
             synth.CubeSpec(96, 80, 70, seed=77, sources=synth.SourcePop(6, 3, 50, True, 1, 8, 2, 20))]
    vols = [synth.cube(s) for s in specs]
    cubes = [r.upload(vols[0], "f32"), r.upload(vols[1], "f16")]
    tf = synth.ramp_tf(256, 1.0)
    r.set_transfer_function(tf, 3.0, 20.0)
    r.set_noise_clip(3.0, 1.0)
    yield r, specs, vols, cubes, tf
    r.server_stop()
    r.close()
    torch.cuda.synchronize()


def make_requests(r, specs, cubes, seed):
    rng = np.random.default_rng(seed)
    sizes = [(256, 256), (100, 37), (512, 512), (64, 64), (33, 200)]
    reqs, outs, meta = [], [], []
    for i in range(10):
        ci = int(rng.integers(0, 2))
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        mode = "ea" if rng.random() < 0.5 else "mip"
        s = specs[ci]
        cam = synth.orbit_camera(s.nx, s.ny, s.nz, float(rng.uniform(0, 6.28)), float(rng.uniform(-0.7, 0.7)))
        out = r.output(W, H, mode)
        out.fill_(math.nan)
        reqs.append(r.request(cubes[ci], cam, W, H, out, mode=mode, clip=3.0))
        outs.append(out)
        meta.append((ci, W, H, mode, cam))
    return reqs, outs, meta


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("graphs", [0, 1])
def test_alone_vs_mix_bit_identical(env, graphs):
    r, specs, vols, cubes, tf = env
    r.server_start(max_batch_requests=64, max_batch_tiles=96, max_inflight=2, use_graphs=graphs)
    try:
        reqs, outs, meta = make_requests(r, specs, cubes, seed=5)
        alone = []
        for q, o in zip(reqs, outs):
            t = r.submit(q)
            lat = r.wait(t, timeout_s=60)
            assert lat >= 0
            alone.append(to_np(o).copy())
            o.fill_(math.nan)
        # the same requests all at once: they share launches and split into tile ranges
        tickets = [r.submit(q) for q in reqs]
        lats = [r.wait(t, timeout_s=60) for t in tickets]
        assert all(l >= 0 for l in lats)
        for a, o in zip(alone, outs):
            b = to_np(o)
            assert not np.isnan(b).any()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    finally:
        r.server_stop()


def test_graph_replays_match_direct_launches(env):
    import torch
    r, specs, vols, cubes, tf = env
    reqs, outs, meta = make_requests(r, specs, cubes, seed=9)
    # reference: direct batched launch, no graphs
    r.render_batch(reqs)
    ref = [to_np(o).copy() for o in outs]
    r.server_start(max_batch_requests=64, max_batch_tiles=4096, max_inflight=1, use_graphs=1)
    try:
        for rep in range(4):
            for o in outs:
                o.fill_(math.nan)
            # eager work between replays
            x = torch.randn(1 << 20, device="cuda")
            _ = (x * 2.0).sum().item()
            tickets = [r.submit(q) for q in reqs]
            for t in tickets:
                r.wait(t, timeout_s=60)
            for a, o in zip(ref, outs):
                assert np.array_equal(a.view(np.uint32), to_np(o).view(np.uint32)), rep
    finally:
        r.server_stop()


def test_served_images_match_renderer_and_reference(env):
    r, specs, vols, cubes, tf = env
    reqs, outs, meta = make_requests(r, specs, cubes, seed=13)
    r.server_start(max_batch_requests=64, max_batch_tiles=256, max_inflight=2, use_graphs=1)
    try:
        tickets = [r.submit(q) for q in reqs]
        for t in tickets:
            r.wait(t, timeout_s=60)
    finally:
        r.server_stop()
    for (ci, W, H, mode, cam), o in list(zip(meta, outs))[:4]:
        served = to_np(o)
        r.set_camera(cam)
        single = to_np(r.render(cubes[ci], W, H, mode=mode))
        assert np.array_equal(served.view(np.uint32), single.view(np.uint32))
        wl = synth.Workload("serve", specs[ci], W, H, v0=3.0, v1=20.0, clip_k=3.0)
        vol = vols[ci]
        if ci == 1:  # float16 storage: the reference reads the decoded codes
            vol = oracle.decode_bits(oracle.to_f16_bits(vol), oracle.F16)
        px = synth.pixel_subset(ci + 3, W, H, 300)
        ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, mode, "trilinear", pixels=px)
        got = served[px[:, 1], px[:, 0]]
        if mode == "ea":
            compare_ea(got, ref["values"], TOL_F32, ref["flags"])
        else:
            compare_mip(got, ref["values"], TOL_F32, ref["flags"], ref.get("bounds"),
                        clip=wl.clip_k)


def test_new_skip_key_first_use_across_slots(env):
    """The first requests for a (cube, transfer function, clip) key that has no
    skip mask yet, split into tile ranges over three inflight slots (separate
    streams), read the mask only once it is built: the served images equal the
    same views rendered with skipping off, bit for bit."""
    r, specs, vols, cubes, tf = env
    s = specs[1]
    cams = [synth.orbit_camera(s.nx, s.ny, s.nz, 0.4 + 1.7 * i, 0.3 - 0.2 * i) for i in range(3)]
    modes = ["ea", "mip", "ea"]
    clip = 3.37  # used by no other test: its skip mask does not exist yet
    outs = [r.output(512, 512, m) for m in modes]
    for o in outs:
        o.fill_(math.nan)
    reqs = [r.request(cubes[1], c, 512, 512, o, mode=m, clip=clip) for c, o, m in zip(cams, outs, modes)]
    r.server_start(max_batch_requests=8, max_batch_tiles=64, max_inflight=3, use_graphs=0)
    try:
        tickets = [r.submit(q) for q in reqs]
        for t in tickets:
            assert r.wait(t, timeout_s=60) >= 0
    finally:
        r.server_stop()
    for c, o, m in zip(cams, outs, modes):
        served = to_np(o)
        assert not np.isnan(served).any()
        r.set_camera(c)
        r.set_noise_clip(clip, 1.0)
        plain = to_np(r.render(cubes[1], 512, 512, mode=m, use_skip=False))
        r.set_noise_clip(3.0, 1.0)
        assert np.array_equal(served.view(np.uint32), plain.view(np.uint32)), m


def test_server_state_errors(env):
    from paper_1001_2049_amd import vr
    r, specs, vols, cubes, tf = env
    out = r.output(16, 16, "mip")
    cam = synth.orbit_camera(64, 64, 128, 0.3, 0.2)
    q = r.request(cubes[0], cam, 16, 16, out, mode="mip")
    with pytest.raises(vr.VRError) as e:
        r.submit(q)
    assert e.value.status == vr.VR_ESTATE
    r.server_start(max_batch_requests=8, max_batch_tiles=1, max_inflight=1, use_graphs=0)
    try:
        big = r.output(512, 512, "ea")
        qs = [r.request(cubes[0], cam, 512, 512, big, mode="ea") for _ in range(4)]
        ts = [r.submit(x) for x in qs]
        # a cube with queued requests cannot be released
        with pytest.raises(vr.VRError) as e:
            r.release(cubes[0])
        assert e.value.status == vr.VR_EBUSY
        for t in ts:
            r.wait(t, timeout_s=120)
        with pytest.raises(vr.VRError) as e:
            r.wait(ts[0])
        assert e.value.status == vr.VR_ENOTFOUND
    finally:
        r.server_stop()
