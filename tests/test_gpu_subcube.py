"""Sub-cube partial images and their integration (paper Sec. 3.1, process
steps 1, 4 and 5): the one-GPU part of sort-last compositing.

Checks that (1) each partial (voxel planes [lo, hi) along an axis, on the
whole cube's lattice) matches the FP64 reference's partial of the same window,
pixels with a sample on a window edge excepted; (2) their sample counts
partition every ray; (3) the "over" composite of EA partials in visibility
order and the maximum of MIP partials match the reference's whole image and
the renderer's own whole image; (4) out-of-range planes are refused."""
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


@pytest.fixture(scope="module")
def scene():
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    spec = synth.CubeSpec(70, 64, 150, seed=4040, sources=synth.SourcePop(8, 4, 30, True, 1.5, 6, 2, 20))
    vol = synth.cube(spec)
    cube = r.upload(vol, "f32")
    tf = synth.ramp_tf(256, 1.0)
    r.set_transfer_function(tf, 3.0, 30.0)
    r.set_noise_clip(3.0, 1.0)
    yield r, spec, vol, cube, tf
    r.close()


def windows(n, cuts):
    edges = [0] + list(cuts) + [n]
    return list(zip(edges[:-1], edges[1:]))


@pytest.mark.parametrize("axis,cuts,cam_kind", [(2, (32, 64, 100), "below"), (2, (37, 90), "orbit"),
                                                (0, (20, 41), "orbit"), (1, (1, 31, 63), "orbit")])
@pytest.mark.parametrize("mode", ["ea", "mip"])
def test_partials_and_composite(scene, axis, cuts, cam_kind, mode):
    r, spec, vol, cube, tf = scene
    if cam_kind == "below":  # every ray moves up in z
        cam = synth.Camera(eye=(34.0, -40.0, -120.0), target=(34.5, 31.5, 74.5), up=(0.0, 0.0, 1.0),
                           fovy_deg=40.0)
    else:
        cam = synth.orbit_camera(70, 64, 150, 2.1, 0.5)
    r.set_camera(cam)
    W, H = 180, 140
    n_axis = (spec.nx, spec.ny, spec.nz)[axis]
    kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=30.0, clip=3.0, step=0.5, ert=2.0)
    parts, counts = [], []
    for lo, hi in windows(n_axis, cuts):
        img, st = r.render_subcube(cube, W, H, axis, lo, hi, mode=mode, ert=2.0, stats=True)
        got = to_np(img).copy()
        wlo = -np.inf if lo == 0 else lo - 0.5
        whi = np.inf if hi == n_axis else hi - 0.5
        ref = ref_render(vol, kw, cam, W, H, mode, "trilinear", window=(axis, wlo, whi))
        counts.append(int(ref["n_nominal"].sum()))
        assert st["samples_nominal"] == counts[-1] or np.any(ref["flags"] & oracle.FLAG_WINDOW_AMBIG)
        if mode == "ea":
            info = compare_ea(got, ref["image"], TOL_F32, ref["flags"])
        else:
            floor = ref["image"] == oracle.MIP_BELOW_CLIP
            g_floor = got == np.float32(-3.402823466e38)
            ok = (ref["flags"] & oracle.FLAGS_AMBIGUOUS) == 0
            assert np.array_equal(floor[ok], g_floor[ok])
            keep = ~floor & ~g_floor
            info = compare_mip(np.where(keep, got, 0.0), np.where(keep, ref["image"], 0.0), TOL_F32,
                               np.where(keep, ref["flags"], 0), clip=-np.inf)
        record("subcube %s axis%d [%d,%d) %s" % (mode, axis, lo, hi, cam_kind), info)
        parts.append(img.clone())
    whole_ref = ref_render(vol, kw, cam, W, H, mode, "trilinear")
    assert sum(counts) == int(whole_ref["n_nominal"].sum())
    comp = to_np(r.composite(parts, axis, W, H, mode=mode))
    whole_gpu = to_np(r.render(cube, W, H, mode=mode, ert=2.0))
    if mode == "ea":
        info = compare_ea(comp, whole_ref["image"], TOL_F32, whole_ref["flags"])
        assert np.max(np.abs(comp - whole_gpu)) <= 2 * TOL_F32
    else:
        info = compare_mip(comp, whole_ref["image"], TOL_F32, whole_ref["flags"],
                           whole_ref.get("bounds"), clip=3.0)
        hit = np.isfinite(whole_gpu)
        assert np.array_equal(hit, np.isfinite(comp))
        assert np.max(np.abs(comp[hit] - whole_gpu[hit]) / np.maximum(1, np.abs(whole_gpu[hit]))) <= 2 * TOL_F32
    record("subcube composite %s axis%d %s" % (mode, axis, cam_kind), info)


def test_top_window_after_mip_renders(scene):
    """Regression: a window that reaches the cube's top face holds samples up
    to the face, whose floor index is the last plane; its slab boxes must
    include that plane's +1 neighbour (the edge copy) rather than read past
    the box, where LDS left by earlier MIP launches (cell bounds of -inf)
    turned weight-0 corners into NaN samples.  MIP frames are rendered first,
    then the top window's EA partial is compared with the reference."""
    r, spec, vol, cube, tf = scene
    for k in range(4):
        r.set_camera(synth.orbit_camera(70, 64, 150, 0.7 + 1.3 * k, 0.4 - 0.25 * k))
        r.render(cube, 180, 140, mode="mip")
    cam = synth.Camera(eye=(34.0, -40.0, -120.0), target=(34.5, 31.5, 74.5), up=(0.0, 0.0, 1.0),
                       fovy_deg=40.0)
    r.set_camera(cam)
    W, H = 180, 140
    img, st = r.render_subcube(cube, W, H, 2, 100, 150, mode="ea", ert=2.0, stats=True)
    got = to_np(img)
    assert np.isfinite(got).all()
    kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=30.0, clip=3.0, step=0.5, ert=2.0)
    ref = ref_render(vol, kw, cam, W, H, "ea", "trilinear", window=(2, 99.5, np.inf))
    info = compare_ea(got, ref["image"], TOL_F32, ref["flags"])
    record("subcube ea top window after mip", info)


def test_subcube_argument_errors(scene):
    from paper_1001_2049_amd import vr
    r, spec, vol, cube, tf = scene
    for axis, lo, hi in [(3, 0, 10), (2, -1, 10), (2, 10, 10), (2, 0, 151)]:
        with pytest.raises(vr.VRError) as e:
            r.render_subcube(cube, 16, 16, axis, lo, hi, mode="mip")
        assert e.value.status == vr.VR_EINVAL
