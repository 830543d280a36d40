"""C interface on the host: the library loads, exports every declared symbol, and
validates arguments (status codes, error text) before any device call.  Uses a
host-only context (device -1), so no GPU is needed."""
import ctypes
import math

import numpy as np
import pytest

from paper_1001_2049_amd import vr


@pytest.fixture(scope="module")
def L():
    return vr.lib()


@pytest.fixture
def ctx(L):
    h = ctypes.c_void_p()
    assert L.vr_create(-1, 0, None, ctypes.byref(h)) == vr.VR_OK
    yield h
    assert L.vr_destroy(h) == vr.VR_OK


def good_camera():
    c = vr.vr_camera()
    c.ortho = 0
    for a, (e, t, u) in enumerate(zip((100.0, 20.0, 30.0), (10.0, 20.0, 30.0), (0.0, 0.0, 1.0))):
        c.eye[a], c.target[a], c.up[a] = e, t, u
    c.fovy_deg = 60.0
    return c


def test_every_declared_function_is_exported(L):
    names = vr.header_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vr._SIGNATURES), "binding and header disagree"
    assert L.vr_version().startswith(b"vr-mi355x")


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(vr.vr_camera) == 8 + 9 * 8 + 3 * 8
    assert ctypes.sizeof(vr.vr_render_params) == 32
    assert ctypes.sizeof(vr.vr_request) == 16 + ctypes.sizeof(vr.vr_camera) + 32 + 8


def test_create_rejects_bad_arguments(L):
    h = ctypes.c_void_p()
    assert L.vr_create(-2, 0, None, ctypes.byref(h)) == vr.VR_EINVAL
    assert L.vr_create(-1, 0, None, None) == vr.VR_EINVAL
    assert L.vr_destroy(None) == vr.VR_EINVAL
    assert b"NULL" in L.vr_last_error()


def test_transfer_function_validation(L, ctx):
    good = np.tile(np.array([0.5, 0.5, 0.5, 1.0], np.float32), (8, 1))
    assert L.vr_set_transfer_function(ctx, good.ctypes.data, 8, 0.0, 1.0) == vr.VR_OK
    assert L.vr_set_transfer_function(ctx, good.ctypes.data, 1, 0.0, 1.0) == vr.VR_EINVAL
    assert L.vr_set_transfer_function(ctx, good.ctypes.data, 8, 1.0, 1.0) == vr.VR_EINVAL
    assert L.vr_set_transfer_function(ctx, good.ctypes.data, 8, 0.0, math.inf) == vr.VR_EINVAL
    assert L.vr_set_transfer_function(ctx, None, 8, 0.0, 1.0) == vr.VR_EINVAL
    bad = good.copy()
    bad[3, 3] = -0.1
    assert L.vr_set_transfer_function(ctx, bad.ctypes.data, 8, 0.0, 1.0) == vr.VR_EINVAL
    assert b"extinction" in L.vr_last_error()
    bad = good.copy()
    bad[2, 1] = np.nan
    assert L.vr_set_transfer_function(ctx, bad.ctypes.data, 8, 0.0, 1.0) == vr.VR_EINVAL
    t = ctypes.c_int32()
    assert L.vr_tf_create(ctx, good.ctypes.data, 8, 0.0, 1.0, ctypes.byref(t)) == vr.VR_OK
    assert t.value > 0
    assert L.vr_tf_release(ctx, t.value) == vr.VR_OK
    assert L.vr_tf_release(ctx, t.value) == vr.VR_ENOTFOUND


def test_camera_validation(L, ctx):
    c = good_camera()
    assert L.vr_set_camera(ctx, ctypes.byref(c)) == vr.VR_OK
    c2 = good_camera()
    c2.up[0], c2.up[1], c2.up[2] = 1.0, 0.0, 0.0  # parallel to the view direction
    assert L.vr_set_camera(ctx, ctypes.byref(c2)) == vr.VR_EINVAL
    assert b"parallel" in L.vr_last_error()
    for fov in (0.0, 180.0, -5.0, math.nan):
        c3 = good_camera()
        c3.fovy_deg = fov
        assert L.vr_set_camera(ctx, ctypes.byref(c3)) == vr.VR_EINVAL
    c4 = good_camera()
    c4.ortho, c4.ortho_w, c4.ortho_h = 1, 10.0, 0.0
    assert L.vr_set_camera(ctx, ctypes.byref(c4)) == vr.VR_EINVAL
    c4.ortho_h = 5.0
    assert L.vr_set_camera(ctx, ctypes.byref(c4)) == vr.VR_OK
    c5 = good_camera()
    c5.eye[2] = math.inf
    assert L.vr_set_camera(ctx, ctypes.byref(c5)) == vr.VR_EINVAL
    assert L.vr_set_camera(ctx, None) == vr.VR_EINVAL


def test_noise_clip_validation(L, ctx):
    assert L.vr_set_noise_clip(ctx, 3.0, 1.0) == vr.VR_OK
    assert L.vr_set_noise_clip(ctx, -math.inf, 1.0) == vr.VR_OK
    assert L.vr_set_noise_clip(ctx, 3.0, 0.0) == vr.VR_EINVAL
    assert L.vr_set_noise_clip(ctx, math.nan, 1.0) == vr.VR_EINVAL
    assert L.vr_set_noise_clip(ctx, math.inf, 1.0) == vr.VR_EINVAL


def test_render_argument_order_and_state(L, ctx):
    p = vr.make_params(64, 64)
    out = ctypes.c_void_p(0x1000)
    bad = vr.make_params(0, 64)
    assert L.vr_render(ctx, 1, ctypes.byref(bad), out, None, None) == vr.VR_EINVAL
    for field, val in (("step", 0.0), ("step", math.nan), ("ert_alpha", 0.0), ("mode", 7),
                       ("interp", 3), ("use_skip", 2), ("height", 16385)):
        q = vr.make_params(64, 64)
        setattr(q, field, val)
        assert L.vr_render(ctx, 1, ctypes.byref(q), out, None, None) == vr.VR_EINVAL, field
    assert L.vr_render(ctx, 1, ctypes.byref(p), None, None, None) == vr.VR_EINVAL
    # no camera yet
    assert L.vr_render(ctx, 1, ctypes.byref(p), out, None, None) == vr.VR_ESTATE
    c = good_camera()
    L.vr_set_camera(ctx, ctypes.byref(c))
    # EA needs a transfer function
    assert L.vr_render(ctx, 1, ctypes.byref(p), out, None, None) == vr.VR_ESTATE
    mip = vr.make_params(64, 64, mode="mip")
    assert L.vr_render(ctx, 1, ctypes.byref(mip), out, None, None) == vr.VR_ENOTFOUND
    assert L.vr_cube_release(ctx, 1) == vr.VR_ENOTFOUND
    info = vr.vr_cube_info()
    assert L.vr_cube_get_info(ctx, 5, ctypes.byref(info)) == vr.VR_ENOTFOUND


def test_upload_validation_and_host_only_context(L, ctx):
    a = np.zeros((4, 4, 4), np.float32)
    cube = ctypes.c_int32()
    P = a.ctypes.data
    assert L.vr_cube_upload(ctx, P, 0, 0, 1, 4, 4, 0, 1.0, None, ctypes.byref(cube)) == vr.VR_EINVAL
    assert L.vr_cube_upload(ctx, P, 0, 0, 4, 4, 4, 9, 1.0, None, ctypes.byref(cube)) == vr.VR_EINVAL
    assert L.vr_cube_upload(ctx, P, 0, 0, 4, 4, 4, 0, 0.0, None, ctypes.byref(cube)) == vr.VR_EINVAL
    assert L.vr_cube_upload(ctx, P, 1, 0, 4, 4, 4, 0, 1.0, None,
                            ctypes.byref(cube)) == vr.VR_EUNSUPPORTED
    assert L.vr_cube_upload(ctx, None, 0, 0, 4, 4, 4, 0, 1.0, None,
                            ctypes.byref(cube)) == vr.VR_EINVAL
    assert L.vr_cube_upload(ctx, P, 0, 0, 4, 4, 4, 0, 1.0, None, ctypes.byref(cube)) == vr.VR_EDEVICE
    assert b"host-only" in L.vr_last_error()


def test_batch_validation(L, ctx):
    assert L.vr_render_batch(ctx, None, -1, None, None) == vr.VR_EINVAL
    assert L.vr_render_batch(ctx, None, 0, None, None) == vr.VR_OK  # empty batch: no-op
    r = vr.vr_request()
    r.cube = 42
    r.camera = good_camera()
    r.params = vr.make_params(32, 32, mode="mip")
    r.out_dev = 0x1000
    arr = (vr.vr_request * 1)(r)
    assert L.vr_render_batch(ctx, arr, 1, None, None) == vr.VR_ENOTFOUND
    assert b"request 0" in L.vr_last_error()
    r.params.width = -3
    arr = (vr.vr_request * 1)(r)
    assert L.vr_render_batch(ctx, arr, 1, None, None) == vr.VR_EINVAL


def test_last_error_is_per_thread(L, ctx):
    import threading
    assert L.vr_set_noise_clip(ctx, 3.0, -1.0) == vr.VR_EINVAL
    main_msg = L.vr_last_error()
    seen = {}

    def other():
        h = ctypes.c_void_p()
        seen["create"] = L.vr_create(-7, 0, None, ctypes.byref(h))
        seen["msg"] = L.vr_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["create"] == vr.VR_EINVAL
    assert seen["msg"] != main_msg
    assert L.vr_last_error() == main_msg


def test_register_validation_and_memory_stats(L, ctx):
    """vr_cube_register validates like vr_cube_upload before touching a device;
    a host-only context keeps no cubes; memory statistics start empty."""
    vol = np.zeros((4, 4, 4), np.float32)
    out = ctypes.c_int32(7)
    p = vol.ctypes.data
    assert L.vr_cube_register(ctx, None, vr.VR_F32, 4, 4, 4, vr.VR_F32, 1.0, ctypes.byref(out)) == vr.VR_EINVAL
    assert out.value == 7 or out.value == 0
    assert L.vr_cube_register(ctx, p, vr.VR_F32, 1, 4, 4, vr.VR_F32, 1.0, ctypes.byref(out)) == vr.VR_EINVAL
    assert L.vr_cube_register(ctx, p, vr.VR_F32, 4, 4, 4, 7, 1.0, ctypes.byref(out)) == vr.VR_EINVAL
    assert L.vr_cube_register(ctx, p, vr.VR_F16, 4, 4, 4, vr.VR_BF16, 1.0,
                              ctypes.byref(out)) == vr.VR_EUNSUPPORTED
    assert L.vr_cube_register(ctx, p, vr.VR_F32, 4, 4, 4, vr.VR_F32, 0.0, ctypes.byref(out)) == vr.VR_EINVAL
    assert L.vr_cube_register(ctx, p, vr.VR_F32, 4, 4, 4, vr.VR_F32, 1.0, ctypes.byref(out)) == vr.VR_EDEVICE
    assert out.value == 0
    m = vr.vr_memory_stats()
    assert L.vr_get_memory_stats(ctx, ctypes.byref(m)) == vr.VR_OK
    assert m.as_dict() == {k: 0 for k, _ in vr.vr_memory_stats._fields_}
    assert L.vr_get_memory_stats(ctx, None) == vr.VR_EINVAL


def test_progressive_and_subcube_validation(L, ctx):
    """vr_render_progressive and vr_render_subcube reject bad arguments before any
    device work; a host-only context cannot render.  The progressive info
    struct matches the header's layout."""
    assert ctypes.sizeof(vr.vr_progressive_info) == 4 + 4 + 4 + 4 + 8 + 4 + 4
    p = vr.make_params(64, 48)
    info = vr.vr_progressive_info()
    out = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails first
    prog = L.vr_render_progressive
    assert prog(None, 1, ctypes.byref(p), 1.0, 3, out, None, ctypes.byref(info)) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), 1.0, 3, out, None, None) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), 1.0, 3, None, None, ctypes.byref(info)) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), 1.0, 5, out, None, ctypes.byref(info)) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), 1.0, -1, out, None, ctypes.byref(info)) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), math.nan, 3, out, None, ctypes.byref(info)) == vr.VR_EINVAL
    bad = vr.make_params(64, 48, step=0.0)
    assert prog(ctx, 1, ctypes.byref(bad), 1.0, 3, out, None, ctypes.byref(info)) == vr.VR_EINVAL
    assert prog(ctx, 1, ctypes.byref(p), 1.0, 3, out, None, ctypes.byref(info)) == vr.VR_EDEVICE
    assert info.level == 0 and info.converged == 0 and info.level_cube == 0
    sub = L.vr_render_subcube
    for axis in (-1, 3):
        assert sub(ctx, 1, ctypes.byref(p), axis, 0, 4, out, None, None) == vr.VR_EINVAL
    assert sub(ctx, 1, ctypes.byref(bad), 2, 0, 4, out, None, None) == vr.VR_EINVAL
