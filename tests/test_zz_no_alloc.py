"""The allocation-free render entry point (vr_render_noalloc), called through
the C interface: for callers that cannot allocate device memory (code under
graph capture, tight serving loops).  Its images must equal vr_render's bit
for bit, on two calls in a row with the second image smaller, and it must
refuse what it cannot do without allocating."""
import ctypes
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_render_matches_render_twice():
    import torch

    from paper_1001_2049_amd import Renderer, vr
    L = vr.lib()
    r = Renderer(0)
    try:
        spec = synth.CubeSpec(72, 64, 90, seed=55, sources=synth.SourcePop(5, 4, 30, True, 1.5, 5, 2, 12))
        vol = synth.cube(spec)
        cube = r.upload(vol, "f32")
        tf = synth.ramp_tf(256, 1.0)
        r.set_transfer_function(tf, 3.0, 30.0)
        r.set_noise_clip(3.0, 1.0)
        stream = torch.cuda.current_stream()
        sp = ctypes.c_void_p(stream.cuda_stream)
        for k, (W, H, mode, th) in enumerate([(300, 200, "ea", 0.5), (96, 40, "ea", 1.7),
                                              (128, 90, "mip", 2.4), (40, 33, "mip", 0.2)]):
            cam = synth.orbit_camera(72, 64, 90, th, 0.35)
            r.set_camera(cam)
            want = r.render(cube, W, H, mode=mode)  # also prepares the skip mask on this stream
            got = r.output(W, H, mode)
            got.fill_(math.nan)
            p = vr.make_params(W, H, mode)
            st = L.vr_render_noalloc(r.ctx, cube, ctypes.byref(p), ctypes.c_void_p(got.data_ptr()), sp)
            assert st == vr.VR_OK, vr.last_error()
            torch.cuda.synchronize()
            a, b = want.cpu().numpy(), got.cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (k, W, H, mode)
        # beyond the fixed scratch: refused, nothing launched
        p = vr.make_params(16384, 16384, "mip")
        big = ctypes.c_void_p(got.data_ptr())
        assert L.vr_render_noalloc(r.ctx, cube, ctypes.byref(p), big, sp) == vr.VR_EINVAL
        assert b"scratch" in L.vr_last_error()
        # a state whose skip mask was never prepared: refused
        r.set_noise_clip(3.5, 1.0)
        p = vr.make_params(40, 33, "mip")
        assert L.vr_render_noalloc(r.ctx, cube, ctypes.byref(p), big, sp) == vr.VR_ESTATE
        r.release(cube)
    finally:
        r.close()
