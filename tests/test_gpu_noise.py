"""Noise-aware form on the GPU: per-channel robust noise estimates and
rendering in units of each channel's noise (the paper's attention to data of
low signal-to-noise ratio, abstract and Sec. 2).

Checks that (1) the device's per-channel lower medians and MADs equal the
FP64 reference's, rounded once to float32 (they are order statistics: exact),
for host and device sources and ragged channel sizes, and sigma agrees to
float32 rounding; (2) a cube with a frequency-dependent noise level, stored
in units of its estimated noise, renders (EA and MIP, float32 and float16
storage) as the FP64 reference renders the same cube scaled by its own
estimates; (3) skipping stays bit-invisible on the scaled cube."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_16, TOL_F32, compare_ea, compare_mip, record, ref_render
from oracle import noise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def band():
    spec = synth.CubeSpec(96, 88, 72, seed=4321,
                          sources=synth.SourcePop(10, 4.0, 40.0, True, 1.5, 5.0, 2.0, 15.0))
    prof = synth.band_noise_profile(72)
    vol = synth.cube_profiled(spec, prof)
    return spec, prof, vol


def check_stats(got, vol):
    med, mad, sig = got
    rmed, rmad, rsig = noise.channel_stats(vol)
    assert np.array_equal(med, rmed.astype(np.float32))
    assert np.array_equal(mad, rmad.astype(np.float32))
    assert np.all(np.abs(sig.astype(np.float64) - rsig) <= 2.0 ** -23 * np.abs(rsig) + 1e-30)


@pytest.mark.parametrize("on_device", [False, True])
def test_channel_noise_matches_reference(R, band, on_device):
    import torch
    spec, prof, vol = band
    src = torch.from_numpy(vol).cuda() if on_device else vol
    got = R.estimate_channel_noise(src)
    check_stats(got, vol)
    # the estimate follows the generator's noise profile (sources in the
    # upper channels bias a robust estimate upwards by up to ~15 % here)
    assert np.max(np.abs(got[2] / prof - 1.0)) < 0.2
    assert np.median(np.abs(got[2] / prof - 1.0)) < 0.05


@pytest.mark.parametrize("shape", [(3, 1, 1), (2, 5, 7), (5, 2, 2), (4, 33, 65)])
def test_channel_noise_ragged_and_degenerate(R, shape):
    rng = np.random.default_rng(sum(shape))
    vol = rng.standard_normal(shape).astype(np.float32)
    vol[0, 0, 0] = -0.0
    if shape[1] * shape[2] > 4:
        vol[1] = 2.5  # a constant channel: MAD 0
    check_stats(R.estimate_channel_noise(vol), vol)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_scaled_cube_renders_like_reference(R, band, storage):
    spec, prof, vol = band
    med, mad, sig = R.estimate_channel_noise(vol)
    div = np.where(sig > 0, sig, np.float32(1.0)).astype(np.float32)
    cube = R.upload_scaled(vol, div, storage)
    try:
        _, _, rsig = noise.channel_stats(vol)
        scaled = noise.scaled_cube(vol, noise.scale_divisors(rsig))
        tf = synth.ramp_tf(256, 1.0)
        R.set_transfer_function(tf, 3.0, 30.0)
        R.set_noise_clip(3.0, 1.0)
        kw = dict(tf=tf.astype(np.float64), v0=3.0, v1=30.0, clip=3.0, step=0.5,
                  ert=float(np.float32(0.99)))
        tol = TOL_F32 if storage == "f32" else TOL_16
        extra = {} if storage == "f32" else dict(amb_ert=TOL_16, amb_clip=TOL_16)
        for vi, (th, ph) in enumerate([(0.4, 0.3), (2.2, -0.5)]):
            cam = synth.orbit_camera(spec.nx, spec.ny, spec.nz, th, ph)
            R.set_camera(cam)
            for mode in ("ea", "mip"):
                img = R.render(cube, 160, 128, mode=mode)
                noskip = R.render(cube, 160, 128, mode=mode, use_skip=False)
                import torch
                torch.cuda.synchronize()
                got, ns = img.cpu().numpy(), noskip.cpu().numpy()
                assert np.array_equal(got.view(np.uint32), ns.view(np.uint32))
                ref = ref_render(scaled, kw, cam, 160, 128, mode, "trilinear", **extra)
                if mode == "ea":
                    info = compare_ea(got, ref["image"], tol, ref["flags"],
                                      max_ambiguous_frac=0.01 if storage == "f32" else 0.05)
                else:
                    info = compare_mip(got, ref["image"], tol, ref["flags"], ref.get("bounds"),
                                       clip=3.0, amb_clip=1e-4 if storage == "f32" else TOL_16)
                record("noise-scaled %s view%d %s" % (storage, vi, mode), info)
    finally:
        R.release(cube)


def test_scaled_upload_rejects_bad_divisors(R, band):
    from paper_1001_2049_amd import vr
    spec, prof, vol = band
    d = np.ones(spec.nz, np.float32)
    d[5] = 0.0
    with pytest.raises(vr.VRError) as e:
        R.upload_scaled(vol, d)
    assert e.value.status == vr.VR_EINVAL
    d[5] = math.nan
    with pytest.raises(vr.VRError) as e:
        R.upload_scaled(vol, d)
    assert e.value.status == vr.VR_EINVAL


def test_progressive_levels_of_a_scaled_cube(R, band):
    """A cube stored in units of each channel's noise (the reference's robust
    sigma as divisors) renders its progressive coarse level as the method on
    the block means of those normalised values, with the one k-sigma clip."""
    import torch
    from oracle import levels
    spec, prof, vol = band
    _, _, rsig = noise.channel_stats(vol)
    div = noise.scale_divisors(rsig).astype(np.float32)
    cube = R.upload_scaled(vol, div, "f32")
    try:
        # the stored values: each voxel divided by its channel's divisor in float32
        stored = (vol.astype(np.float32) / div[:, None, None]).astype(np.float32)
        tf = synth.ramp_tf(256, 1.0)
        R.set_transfer_function(tf, 3.0, 30.0)
        R.set_noise_clip(3.0, 1.0)
        cam = synth.orbit_camera(spec.nx, spec.ny, spec.nz, 0.8, 0.35)
        R.set_camera(cam)
        W, H = 150, 130
        out = R.output(W, H, "ea")
        info = R.render_progressive(cube, W, H, out, budget_ms=1e-6, max_level=1, mode="ea")
        assert info["level"] == 1 and info["level_cube"] == 1
        torch.cuda.synchronize()
        low = out.cpu().numpy()[::2, ::2]
        wl, hl = levels.level_size(W, H, 1)
        kw = dict(tf=levels.level_tf(tf, 1), v0=3.0, v1=30.0, clip=3.0, step=0.5,
                  ert=float(np.float32(0.99)))
        ref = ref_render(levels.level_volume(stored, 1), kw, levels.level_camera(cam, 1), wl, hl,
                         "ea", "trilinear")
        record("scaled cube progressive level 1", compare_ea(low, ref["image"], TOL_F32, ref["flags"]))
    finally:
        R.release(cube)
