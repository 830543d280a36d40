"""GPU renderer vs the FP64 reference, element by element, through the C interface.

Sizes span several 16x16-pixel workgroup tiles (256 threads), several 32^3 bricks and 8^3 skip
cells, and ragged edges (image and cube sizes that are not multiples of the
tile/brick/cell sizes).  Tolerances: max per-channel absolute error 1e-5 for
float32 storage (RGBA in [0,1]); MIP values within 1e-5 * max(1, |m|);
axis-aligned orthographic MIP with nearest sampling bit-exact.  Pixels the
reference flags as ambiguous (a quantity within a hair of a decision
threshold, where several results are correct) are counted and bounded
separately.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_F32, compare_ea, compare_mip, record, ref_render, set_state, wl_kwargs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def tiny():
    wl = synth.tiny()
    vol = synth.cube(wl.cube)
    return wl, vol, synth.ramp_tf(256, wl.kappa_max)


@pytest.fixture(scope="module")
def tiny_cube(R, tiny):
    wl, vol, tf = tiny
    return R.upload(vol, "f32")


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------------------
# closed form on the GPU: axis-aligned orthographic MIP, nearest == column max
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("axis", ["z", "x", "y"])
@pytest.mark.parametrize("clip", [True, False])
def test_axis_mip_nearest_bit_exact(R, tiny, tiny_cube, axis, clip):
    wl, vol, tf = tiny
    W = H = 256
    cam = synth.axis_camera(64, 64, 128, axis, W, H)
    set_state(R, wl, tf, cam, clip=clip)
    img = to_np(R.render(tiny_cube, W, H, mode="mip", interp="nearest", step=wl.step))
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, "mip", "nearest",
                     clip=wl.clip_k if clip else -math.inf)
    assert np.array_equal(img.astype(np.float64), ref["image"])


@pytest.mark.parametrize("view", ["z", "orbit0", "orbit1"])
@pytest.mark.parametrize("interp", ["trilinear", "nearest"])
def test_tiny_mip(R, tiny, tiny_cube, view, interp):
    wl, vol, tf = tiny
    W, H = 256, 200
    cam = (synth.axis_camera(64, 64, 128, "z", W, H) if view == "z" else
           synth.orbit_camera(64, 64, 128, *[(0.4, 0.3), (2.5, -0.7)][int(view[-1])]))
    set_state(R, wl, tf, cam)
    img = to_np(R.render(tiny_cube, W, H, mode="mip", interp=interp, step=wl.step))
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, "mip", interp)
    info = compare_mip(img, ref["image"], TOL_F32 if interp == "trilinear" else 0.0, ref["flags"],
                       ref.get("bounds"), clip=wl.clip_k * wl.cube.sigma)
    record("tiny f32 %dx%d %s mip %s" % (W, H, view, interp), info)


@pytest.mark.parametrize("view", ["z", "x", "orbit0", "orbit1", "orbit2"])
@pytest.mark.parametrize("ert", [0.99, 2.0])
def test_tiny_ea(R, tiny, tiny_cube, view, ert):
    wl, vol, tf = tiny
    W, H = 256, 256
    orbits = [(0.4, 0.3), (2.5, -0.7), (4.0, 1.2)]
    cam = (synth.axis_camera(64, 64, 128, view, W, H) if len(view) == 1 else
           synth.orbit_camera(64, 64, 128, *orbits[int(view[-1])]))
    set_state(R, wl, tf, cam)
    img = to_np(R.render(tiny_cube, W, H, mode="ea", step=wl.step, ert=ert))
    kw = wl_kwargs(wl, tf)
    kw["ert"] = float(np.float32(ert))
    ref = ref_render(vol, kw, cam, W, H, "ea", "trilinear")
    info = compare_ea(img, ref["image"], TOL_F32, ref["flags"])
    record("tiny f32 %dx%d %s ea ert%g" % (W, H, view, ert), info)


def test_tiny_frame_times(R, tiny, tiny_cube):
    """Frame times of the tiny workload's z view (256^2) on the GPU (median of
    the library's own kernel timing over 20 frames) and for the FP64
    reference on all host threads, for EA and both MIP interpolations."""
    import os
    import time
    wl, vol, tf = tiny
    W = H = 256
    cam = synth.axis_camera(64, 64, 128, "z", W, H)
    set_state(R, wl, tf, cam)
    for mode, interp in (("ea", "trilinear"), ("mip", "trilinear"), ("mip", "nearest")):
        ms = []
        for _ in range(20):
            _, st = R.render(tiny_cube, W, H, mode=mode, interp=interp, step=wl.step, stats=True)
            ms.append(st["kernel_ms"])
        t0 = time.perf_counter()
        ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, mode, interp, threads=os.cpu_count())
        t_ref = time.perf_counter() - t0
        nominal = int(ref["n_nominal"].sum())
        assert st["samples_nominal"] == nominal
        record("timing tiny f32 256x256 z %s %s" % (mode, interp),
               {"gpu_ms": float(np.median(ms)), "oracle_ms": t_ref * 1e3, "oracle_threads": os.cpu_count(),
                "samples_nominal": nominal})


def test_tiny_ea_opaque_ert(R, tiny, tiny_cube):
    """A strongly absorbing transfer function: many rays terminate early."""
    wl, vol, _ = tiny
    tf = synth.ramp_tf(256, 8.0)
    W, H = 200, 160
    cam = synth.orbit_camera(64, 64, 128, 1.1, 0.4)
    set_state(R, wl, tf, cam)
    img, st = R.render(tiny_cube, W, H, mode="ea", step=wl.step, ert=0.99, stats=True)
    img = to_np(img)
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, "ea", "trilinear")
    compare_ea(img, ref["image"], TOL_F32, ref["flags"])
    stopped = (ref["flags"] & oracle.FLAG_ERT_STOPPED) > 0
    assert stopped.sum() > 20
    assert st["rays_ert"] > 0
    assert st["samples_nominal"] == int(ref["n_nominal"].sum())


# ---------------------------------------------------------------------------
# closed forms on the GPU: constant cube slab law
# ---------------------------------------------------------------------------
def test_constant_cube_slab_law(R):
    N = (40, 36, 50)
    v = 7.3
    vol = np.full(N[::-1], v, dtype=np.float32)
    cube = R.upload(vol, "f32")
    try:
        tf = synth.ramp_tf(256, 0.2)
        v0, v1 = 2.0, 12.0
        R.set_transfer_function(tf, v0, v1)
        R.set_noise_clip(-math.inf, 1.0)
        cam = synth.Camera(eye=(-40.0, 70.0, 90.0), target=(19.5, 17.5, 24.5), up=(0, 0, 1),
                           fovy_deg=40.0)
        R.set_camera(cam)
        W, H = 96, 80
        img = to_np(R.render(cube, W, H, mode="ea", step=0.5, ert=2.0)).astype(np.float64)
        # kappa and rgb of the (float32) table at v, from the table's linear interpolation
        u = (v - v0) / (v1 - v0) * 255
        rows = tf.astype(np.float64)
        k = [np.interp(u, np.arange(256), rows[:, c]) for c in range(4)]
        hit = img[..., 3] > 0
        assert hit.sum() > 1000
        for j, i in zip(*np.nonzero(hit)):
            o, d = oracle.pixel_ray(cam, W, H, i, j)
            ok, t0, t1 = oracle.slab(N[::-1], cam, W, H, o, d)
            assert ok
            A = 1.0 - math.exp(-k[3] * (t1 - t0))
            assert abs(img[j, i, 3] - A) < TOL_F32
            assert max(abs(img[j, i, c] - k[c] * A) for c in range(3)) < TOL_F32
    finally:
        R.release(cube)


# ---------------------------------------------------------------------------
# ragged and degenerate shapes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,img", [((45, 70, 33), (100, 37)), ((2, 2, 2), (7, 5)),
                                       ((33, 9, 65), (1, 1)), ((3, 64, 31), (129, 17))])
@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_ragged_shapes(R, shape, img, mode):
    nx, ny, nz = shape
    spec = synth.CubeSpec(nx, ny, nz, seed=31 + nx, sources=synth.SourcePop(3, 5, 20, False, 1, 4, 1, 4))
    vol = synth.cube(spec)
    cube = R.upload(vol, "f32")
    try:
        tf = synth.ramp_tf(256, 1.0)
        wl = synth.Workload("ragged", spec, img[0], img[1], v0=2.0, v1=15.0, clip_k=2.0)
        W, H = img
        for cam in [synth.orbit_camera(nx, ny, nz, 0.9, 0.5, fovy_deg=50),
                    synth.orbit_camera(nx, ny, nz, 3.9, -1.3, fovy_deg=70, dist_factor=1.2)]:
            set_state(R, wl, tf, cam)
            out = to_np(R.render(cube, W, H, mode=mode, step=0.37, ert=0.99))
            ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, mode, "trilinear", step=float(np.float32(0.37)))
            if mode == "ea":
                compare_ea(out, ref["image"], TOL_F32, ref["flags"])
            else:
                compare_mip(out, ref["image"], TOL_F32, ref["flags"], ref.get("bounds"),
                            clip=wl.clip_k * wl.cube.sigma)
    finally:
        R.release(cube)


@pytest.mark.parametrize("img", [(16384, 3), (5, 16384)])
@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_maximum_image_extents(R, tiny, tiny_cube, img, mode):
    """Images at the largest width and height the interface accepts (16384):
    tile grids of 512 x 1 and 1 x 1024 with ragged last tiles; 600 seeded
    pixels per image, the image's last row and column among them, are
    compared with the reference."""
    wl, vol, tf = tiny
    W, H = img
    cam = synth.orbit_camera(64, 64, 128, 0.4, 0.3, fovy_deg=40)
    set_state(R, wl, tf, cam)
    out = to_np(R.render(tiny_cube, W, H, mode=mode))
    px = np.concatenate([synth.pixel_subset(900 + W, W, H, 600),
                         np.array([[W - 1, H - 1], [W - 1, 0], [0, H - 1]], dtype=np.int64)])
    got = out[px[:, 1], px[:, 0]]
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, W, H, mode, "trilinear", pixels=px)
    if mode == "ea":
        compare_ea(got, ref["values"], TOL_F32, ref["flags"])
    else:
        compare_mip(got, ref["values"], TOL_F32, ref["flags"], ref.get("bounds"),
                    clip=wl.clip_k * wl.cube.sigma)


def test_camera_inside_cube_and_missing_view(R, tiny, tiny_cube):
    wl, vol, tf = tiny
    W, H = 64, 48
    inside = synth.Camera(eye=(30.2, 33.1, 60.7), target=(10.0, 50.0, 100.0), up=(0, 0, 1),
                          fovy_deg=90.0)
    set_state(R, wl, tf, inside)
    img = to_np(R.render(tiny_cube, W, H, mode="ea"))
    ref = ref_render(vol, wl_kwargs(wl, tf), inside, W, H, "ea", "trilinear")
    compare_ea(img, ref["image"], TOL_F32, ref["flags"])
    away = synth.Camera(eye=(500.0, 500.0, 500.0), target=(900.0, 900.0, 900.0), up=(0, 0, 1))
    set_state(R, wl, tf, away)
    img = to_np(R.render(tiny_cube, W, H, mode="mip"))
    assert np.all(np.isneginf(img))
    img = to_np(R.render(tiny_cube, W, H, mode="ea"))
    assert np.all(img == 0.0)


# ---------------------------------------------------------------------------
# invariants: skipping and repetition never change a bit; batch == single
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode,interp", [("ea", "trilinear"), ("mip", "trilinear"),
                                         ("ea", "nearest"), ("mip", "nearest")])
def test_skip_is_bit_invisible(R, tiny, tiny_cube, mode, interp):
    """With the transfer function starting at a 5.5 sigma clip, noise alone
    rarely reaches the clip, most cells are empty and skipping removes work;
    the images with and without it are bit-identical."""
    wl, vol, tf = tiny
    cam = synth.orbit_camera(64, 64, 128, 0.7, 0.2)
    R.set_transfer_function(tf, 5.5, wl.v1)
    R.set_noise_clip(5.5, 1.0)
    R.set_camera(cam)
    a, sa = R.render(tiny_cube, 192, 160, mode=mode, interp=interp, use_skip=True, stats=True)
    b, sb = R.render(tiny_cube, 192, 160, mode=mode, interp=interp, use_skip=False, stats=True)
    c = R.render(tiny_cube, 192, 160, mode=mode, interp=interp, use_skip=True)
    a, b, c = to_np(a), to_np(b), to_np(c)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    assert sa["samples_nominal"] == sb["samples_nominal"]
    assert sa["samples_exec"] < sb["samples_exec"]


def test_batch_equals_single(R, tiny, tiny_cube):
    import torch
    wl, vol, tf = tiny
    set_state(R, wl, tf, synth.orbit_camera(64, 64, 128, 0.0, 0.0))
    reqs, outs, singles = [], [], []
    specs = [("ea", 256, 256, (0.3, 0.2)), ("mip", 100, 37, (1.3, -0.4)), ("ea", 17, 129, (2.0, 0.9)),
             ("mip", 256, 256, (5.0, 0.1)), ("ea", 64, 64, (3.3, -1.0))]
    for mode, W, H, ang in specs:
        cam = synth.orbit_camera(64, 64, 128, *ang)
        out = R.output(W, H, mode)
        reqs.append(R.request(tiny_cube, cam, W, H, out, mode=mode, clip=wl.clip_k))
        outs.append(out)
        R.set_camera(cam)
        singles.append(to_np(R.render(tiny_cube, W, H, mode=mode)))
    stats = R.render_batch(reqs, stats=True)
    for o, s in zip(outs, singles):
        assert np.array_equal(to_np(o).view(np.uint32), s.view(np.uint32))
    assert all(st["samples_nominal"] > 0 for st in stats)
    torch.cuda.synchronize()


def test_batch_request_beyond_one_ordering_run(R, tiny, tiny_cube):
    """A batched request of 32768 tiles (more than one workgroup orders at
    once, so its tiles are ordered in two runs) beside a small request of
    another class: both images equal their single renders bit for bit."""
    import torch
    wl, vol, tf = tiny
    cam = synth.orbit_camera(64, 64, 128, 0.7, 0.35)
    set_state(R, wl, tf, cam)
    big = R.output(4096, 2048, "ea")
    small = R.output(96, 80, "mip")
    R.render_batch([R.request(tiny_cube, cam, 4096, 2048, big, mode="ea", clip=wl.clip_k),
                    R.request(tiny_cube, cam, 96, 80, small, mode="mip", clip=wl.clip_k)])
    single_big = to_np(R.render(tiny_cube, 4096, 2048, mode="ea"))
    single_small = to_np(R.render(tiny_cube, 96, 80, mode="mip"))
    assert np.array_equal(to_np(big).view(np.uint32), single_big.view(np.uint32))
    assert np.array_equal(to_np(small).view(np.uint32), single_small.view(np.uint32))
    torch.cuda.synchronize()


def test_stats_count_nominal_samples(R, tiny, tiny_cube):
    wl, vol, tf = tiny
    cam = synth.orbit_camera(64, 64, 128, 2.2, 0.6)
    set_state(R, wl, tf, cam)
    _, st = R.render(tiny_cube, 128, 96, mode="mip", stats=True)
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, 128, 96, "mip", "trilinear")
    assert st["samples_nominal"] == int(ref["n_nominal"].sum())
    assert st["rays_hit"] == int(((ref["flags"] & oracle.FLAG_HIT) > 0).sum())
    assert st["kernel_ms"] > 0


# ---------------------------------------------------------------------------
# full-size workload in the benchmark's launch configuration, sampled pixels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_full_cube_whole_frames(R, full_workload, mode):
    """512x512x1024 float32 cube, 1024^2 perspective orbit views, skipping on,
    early termination at 0.99, rendered as in the benchmark: two whole frames
    compared pixel by pixel with the reference, and 2000 seeded pixels of a
    third view."""
    wl, vol, tf = full_workload
    cube = R.upload(vol, "f32")
    try:
        kw = wl_kwargs(wl, tf)
        for vi, (th, ph) in enumerate(synth.orbit_angles(wl.extra["camera_seed"], 3)):
            cam = synth.orbit_camera(512, 512, 1024, th, ph)
            set_state(R, wl, tf, cam)
            img, st = R.render(cube, 1024, 1024, mode=mode, stats=True)
            got_img = to_np(img)
            if vi < 2:
                ref = ref_render(vol, kw, cam, 1024, 1024, mode, "trilinear")
                got, want, flags, bnd = got_img, ref["image"], ref["flags"], ref.get("bounds")
                assert st["samples_nominal"] == int(ref["n_nominal"].sum())
            else:
                px = synth.pixel_subset(500 + vi, 1024, 1024, 2000)
                ref = ref_render(vol, kw, cam, 1024, 1024, mode, "trilinear", pixels=px)
                got, want, flags, bnd = (got_img[px[:, 1], px[:, 0]], ref["values"], ref["flags"],
                                         ref.get("bounds"))
            if mode == "ea":
                info = compare_ea(got, want, TOL_F32, flags)
            else:
                info = compare_mip(got, want, TOL_F32, flags, bnd, clip=wl.clip_k)
            record("full f32 1024 view%d %s %s" % (vi, mode, "frame" if vi < 2 else "sampled"), info)
            assert st["samples_exec"] <= st["samples_nominal"]
    finally:
        R.release(cube)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_full_cube_wave_skip_is_bit_invisible(R, full_workload, storage):
    """Full-size cube with the transfer function and clip raised to 4 and 5
    sigma, where under a quarter of most slab boxes' cells are active and the
    waves pass over chunks of 8 samples: images with and without skipping are
    bit-identical (EA and MIP, trilinear and nearest, four orbit views), and
    skipping removes most samples."""
    import torch
    wl, vol, tf = full_workload
    cube = R.upload(vol, storage)
    try:
        for clip in (4.0, 5.0):
            R.set_transfer_function(tf, clip, wl.v1)
            R.set_noise_clip(clip, 1.0)
            for vi, (th, ph) in enumerate(synth.orbit_angles(77, 4)):
                R.set_camera(synth.orbit_camera(512, 512, 1024, th, ph))
                for mode, interp in (("ea", "trilinear"), ("mip", "trilinear"), ("mip", "nearest")):
                    a, sa = R.render(cube, 768, 640, mode=mode, interp=interp, use_skip=True, stats=True)
                    b, sb = R.render(cube, 768, 640, mode=mode, interp=interp, use_skip=False, stats=True)
                    torch.cuda.synchronize()
                    assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (clip, vi, mode, interp)
                    assert sa["samples_nominal"] == sb["samples_nominal"]
                    print("wave skip %s clip %.0f view%d %s/%s: exec %d of %d" % (
                        storage, clip, vi, mode, interp, sa["samples_exec"], sb["samples_exec"]))
                    assert sa["samples_exec"] < 0.75 * sb["samples_exec"], (clip, vi, mode, interp)
    finally:
        R.release(cube)


def test_batch_with_many_fresh_skip_masks(R, tiny, tiny_cube):
    """One batch whose requests need more skip masks on one cube than the cache
    holds (EA and MIP, ten noise clips): every image equals its single render."""
    import torch
    wl, vol, tf = tiny
    R.set_transfer_function(tf, wl.v0, wl.v1)
    cam = synth.orbit_camera(64, 64, 128, 1.3, 0.4)
    reqs, outs, singles = [], [], []
    for q in range(10):
        clip = 2.0 + 0.4 * q
        for mode in ("ea", "mip"):
            out = R.output(96, 80, mode)
            reqs.append(R.request(tiny_cube, cam, 96, 80, out, mode=mode, clip=clip))
            outs.append(out)
    R.render_batch(reqs)
    torch.cuda.synchronize()
    got = [to_np(o).copy() for o in outs]
    R.set_camera(cam)
    for q in range(10):
        R.set_noise_clip(2.0 + 0.4 * q, 1.0)
        for mode in ("ea", "mip"):
            singles.append(to_np(R.render(tiny_cube, 96, 80, mode=mode)).copy())
    for a, b in zip(got, singles):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_large_transfer_function_parity(R, tiny, tiny_cube):
    """A 4096-row transfer function leaves little LDS for slab boxes, so most
    slabs are sampled straight from the brick pool; the image still matches
    the reference, and equals the image a batch launch renders."""
    import torch
    wl, vol, _ = tiny
    tf = synth.ramp_tf(4096, wl.kappa_max)
    cam = synth.orbit_camera(64, 64, 128, 0.4, 0.3)
    R.set_transfer_function(tf, wl.v0, wl.v1)
    R.set_noise_clip(wl.clip_k, 1.0)
    R.set_camera(cam)
    img = to_np(R.render(tiny_cube, 160, 120, mode="ea"))
    ref = ref_render(vol, wl_kwargs(wl, tf), cam, 160, 120, "ea", "trilinear")
    compare_ea(img, ref["image"], TOL_F32, ref["flags"])
    out = R.output(160, 120, "ea")
    R.render_batch([R.request(tiny_cube, cam, 160, 120, out, mode="ea", clip=wl.clip_k)])
    torch.cuda.synchronize()
    assert np.array_equal(img.view(np.uint32), to_np(out).view(np.uint32))


def test_batch_mixing_transfer_function_sizes(R, tiny, tiny_cube):
    """One batch with a 256-row and a 4096-row transfer function (the larger
    table fixes the LDS split of the whole launch, so the small one's slabs
    get smaller box buffers): each image equals its single render bit for
    bit."""
    import torch
    wl, vol, _ = tiny
    small_tf = R.tf_create(synth.ramp_tf(256, wl.kappa_max), wl.v0, wl.v1)
    big_tf = R.tf_create(synth.ramp_tf(4096, wl.kappa_max), wl.v0, wl.v1)
    try:
        cams = [synth.orbit_camera(64, 64, 128, 0.4, 0.3), synth.orbit_camera(64, 64, 128, 2.5, -0.2)]
        outs = [R.output(160, 120, "ea") for _ in cams]
        R.render_batch([R.request(tiny_cube, cams[0], 160, 120, outs[0], mode="ea", clip=wl.clip_k, tf=small_tf),
                        R.request(tiny_cube, cams[1], 160, 120, outs[1], mode="ea", clip=wl.clip_k, tf=big_tf)])
        batch = [to_np(o).copy() for o in outs]
        for tfid, cam, b in zip((small_tf, big_tf), cams, batch):
            single = R.output(160, 120, "ea")
            R.render_batch([R.request(tiny_cube, cam, 160, 120, single, mode="ea", clip=wl.clip_k, tf=tfid)])
            assert np.array_equal(b.view(np.uint32), to_np(single).view(np.uint32))
        torch.cuda.synchronize()
    finally:
        R.tf_release(small_tf)
        R.tf_release(big_tf)


@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_rays_grazing_the_low_faces(R, mode):
    """Rays that cross a cube only within half a voxel of its low x face
    (positions in [-1/2, 0), which read voxel 0), in tiles whose other rays
    lie further out: regression test for slab boxes that left out voxel 0.
    The eye sits below and beside the cube; a z ramp makes every sample's
    height visible in the MIP, and a noisy cube checks EA."""
    ramp = np.arange(150, dtype=np.float32)[:, None, None] * np.ones((1, 64, 70), np.float32)
    spec = synth.CubeSpec(70, 64, 150, seed=4040, sources=synth.SourcePop(8, 4, 30, True, 1.5, 6, 2, 20))
    cam = synth.Camera(eye=(34.0, -40.0, -120.0), target=(34.5, 31.5, 74.5), up=(0.0, 0.0, 1.0),
                       fovy_deg=40.0)
    vol = ramp if mode == "mip" else synth.cube(spec)
    cube = R.upload(vol, "f32")
    try:
        tf = synth.ramp_tf(256, 1.0)
        R.set_transfer_function(tf, 3.0, 30.0)
        R.set_noise_clip(-math.inf if mode == "mip" else 3.0, 1.0)
        R.set_camera(cam)
        got = to_np(R.render(cube, 180, 140, mode=mode))
        kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=30.0, clip=-math.inf if mode == "mip" else 3.0,
                  step=0.5, ert=float(np.float32(0.99)))
        ref = ref_render(vol, kw, cam, 180, 140, mode, "trilinear")
        if mode == "ea":
            compare_ea(got, ref["image"], TOL_F32, ref["flags"])
        else:
            compare_mip(got, ref["image"], TOL_F32, ref["flags"], ref.get("bounds"))
    finally:
        R.release(cube)
