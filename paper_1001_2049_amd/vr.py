"""ctypes binding of the renderer's C interface (include/vr.h).

Argument marshalling only: every step of rendering runs in the HIP library
(libvr.so).  The functions keep the C names; ``Renderer`` is a small
convenience object on top that uses PyTorch for device memory and streams.
Importing this module never falls back to anything: if the library is not
built, ``lib()`` raises.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
import math
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# VR_LIB_PATH selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("VR_LIB_PATH") or os.path.join(HERE, "libvr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vr.h")

VR_OK, VR_EINVAL, VR_ENOMEM, VR_ENOTFOUND, VR_EBUSY, VR_EDEVICE, VR_EUNSUPPORTED, VR_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
VR_F32, VR_F16, VR_BF16 = 0, 1, 2
VR_EA, VR_MIP = 0, 1
VR_NEAREST, VR_TRILINEAR = 0, 1

STATUS_NAMES = {0: "VR_OK", -1: "VR_EINVAL", -2: "VR_ENOMEM", -3: "VR_ENOTFOUND", -4: "VR_EBUSY",
                -5: "VR_EDEVICE", -6: "VR_EUNSUPPORTED", -7: "VR_ESTATE"}


class vr_allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)),
                ("user", ctypes.c_void_p)]


class vr_camera(ctypes.Structure):
    _fields_ = [("ortho", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fovy_deg", ctypes.c_double),
                ("ortho_w", ctypes.c_double), ("ortho_h", ctypes.c_double)]


class vr_render_params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("interp", ctypes.c_int32), ("step", ctypes.c_float),
                ("ert_alpha", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("use_skip", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class vr_stats(ctypes.Structure):
    _fields_ = [("samples_nominal", ctypes.c_uint64), ("samples_exec", ctypes.c_uint64),
                ("rays_hit", ctypes.c_uint64), ("rays_ert", ctypes.c_uint64),
                ("cells_skipped", ctypes.c_uint64), ("kernel_ms", ctypes.c_float),
                ("reserved", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class vr_cube_info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("storage", ctypes.c_int32), ("brick", ctypes.c_int32),
                ("bricks_x", ctypes.c_int32), ("bricks_y", ctypes.c_int32),
                ("bricks_z", ctypes.c_int32), ("cell", ctypes.c_int32),
                ("sigma_scale", ctypes.c_double), ("pool_bytes", ctypes.c_uint64),
                ("brick_stride", ctypes.c_uint64), ("aux_bytes", ctypes.c_uint64),
                ("vmin", ctypes.c_float), ("vmax", ctypes.c_float),
                ("x_chunks", ctypes.c_int32), ("resident", ctypes.c_uint8),
                ("registered", ctypes.c_uint8), ("reserved", ctypes.c_uint16),
                ("pool", ctypes.c_void_p), ("cell_minmax", ctypes.c_void_p)]


class vr_request(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_int32), ("tf", ctypes.c_int32), ("clip", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("camera", vr_camera),
                ("params", vr_render_params), ("out_dev", ctypes.c_void_p)]


class vr_memory_stats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64),
                ("cubes", ctypes.c_uint64), ("resident_cubes", ctypes.c_uint64),
                ("registered_cubes", ctypes.c_uint64), ("uploads", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vr_progressive_info(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("converged", ctypes.c_int32), ("ms", ctypes.c_float),
                ("predicted_ms", ctypes.c_float), ("samples_nominal", ctypes.c_uint64),
                ("level_cube", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vr_server_cfg(ctypes.Structure):
    _fields_ = [("max_batch_requests", ctypes.c_int32), ("max_batch_tiles", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("use_graphs", ctypes.c_int32)]


_lib = None
P = ctypes.c_void_p
S = ctypes.c_int32

_SIGNATURES = {
    "vr_create": (S, [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(vr_allocator),
                      ctypes.POINTER(P)]),
    "vr_destroy": (S, [P]),
    "vr_last_error": (ctypes.c_char_p, []),
    "vr_version": (ctypes.c_char_p, []),
    "vr_cube_upload": (S, [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P,
                           ctypes.POINTER(ctypes.c_int32)]),
    "vr_cube_register": (S, [P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]),
    "vr_get_memory_stats": (S, [P, ctypes.POINTER(vr_memory_stats)]),
    "vr_estimate_channel_noise": (S, [P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, P, P, P, P]),
    "vr_cube_upload_scaled": (S, [P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int32, P, P,
                                  ctypes.POINTER(ctypes.c_int32)]),
    "vr_cube_release": (S, [P, ctypes.c_int32]),
    "vr_cube_get_info": (S, [P, ctypes.c_int32, ctypes.POINTER(vr_cube_info)]),
    "vr_set_transfer_function": (S, [P, P, ctypes.c_int32, ctypes.c_float, ctypes.c_float]),
    "vr_set_noise_clip": (S, [P, ctypes.c_float, ctypes.c_float]),
    "vr_set_camera": (S, [P, ctypes.POINTER(vr_camera)]),
    "vr_render": (S, [P, ctypes.c_int32, ctypes.POINTER(vr_render_params), P, P,
                      ctypes.POINTER(vr_stats)]),
    "vr_render_progressive": (S, [P, ctypes.c_int32, ctypes.POINTER(vr_render_params),
                                  ctypes.c_double, ctypes.c_int32, P, P,
                                  ctypes.POINTER(vr_progressive_info)]),
    "vr_render_subcube": (S, [P, ctypes.c_int32, ctypes.POINTER(vr_render_params), ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, P, P, ctypes.POINTER(vr_stats)]),
    "vr_composite": (S, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]),
    "vr_render_noalloc": (S, [P, ctypes.c_int32, ctypes.POINTER(vr_render_params), P, P]),
    "vr_tf_create": (S, [P, P, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                         ctypes.POINTER(ctypes.c_int32)]),
    "vr_tf_release": (S, [P, ctypes.c_int32]),
    "vr_render_batch": (S, [P, ctypes.POINTER(vr_request), ctypes.c_int32, P,
                            ctypes.POINTER(vr_stats)]),
    "vr_server_start": (S, [P, ctypes.POINTER(vr_server_cfg)]),
    "vr_server_stop": (S, [P]),
    "vr_submit": (S, [P, ctypes.POINTER(vr_request), ctypes.POINTER(ctypes.c_uint64)]),
    "vr_poll": (S, [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "vr_wait": (S, [P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
}


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/vr.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:vr_status|const char\*)\s+(vr_[a-z0-9_]+)\s*\(", text,
                                 flags=re.M)))


def lib():
    """Load libvr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvr.so is not built: run paper_1001_2049_amd/build.py "
                               "(or __graft_entry__.build()) first")
        # PyTorch owns device memory and streams: its HIP runtime must be the one
        # this library binds to (same soname), so it is loaded first
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class VRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


def last_error() -> str:
    return (lib().vr_last_error() or b"").decode()


def check(status: int) -> int:
    if status != VR_OK:
        raise VRError(status, last_error())
    return status


# ---------------------------------------------------------------------------
# helpers to build the C structs
# ---------------------------------------------------------------------------
def make_camera(cam) -> vr_camera:
    """From any object with eye/target/up (3-sequences) and fovy_deg/ortho/ortho_w/ortho_h."""
    c = vr_camera()
    c.ortho = int(bool(getattr(cam, "ortho", False)))
    for a in range(3):
        c.eye[a], c.target[a], c.up[a] = cam.eye[a], cam.target[a], cam.up[a]
    c.fovy_deg = float(getattr(cam, "fovy_deg", 60.0))
    c.ortho_w = float(getattr(cam, "ortho_w", 0.0) or 0.0)
    c.ortho_h = float(getattr(cam, "ortho_h", 0.0) or 0.0)
    return c


def make_params(width, height, mode="ea", interp="trilinear", step=0.5, ert=0.99,
                use_skip=True) -> vr_render_params:
    p = vr_render_params()
    p.mode = {"ea": VR_EA, "mip": VR_MIP}[mode] if isinstance(mode, str) else int(mode)
    p.interp = ({"nearest": VR_NEAREST, "trilinear": VR_TRILINEAR}[interp]
                if isinstance(interp, str) else int(interp))
    p.step = step
    p.ert_alpha = ert
    p.width, p.height = int(width), int(height)
    p.use_skip = int(bool(use_skip))
    return p


STORAGE = {"f32": VR_F32, "f16": VR_F16, "bf16": VR_BF16, VR_F32: VR_F32, VR_F16: VR_F16,
           VR_BF16: VR_BF16}


def torch_allocator(device: int):
    """A vr_allocator that draws device memory from PyTorch's caching allocator."""
    import torch

    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device)
        except Exception:  # noqa: BLE001 - reported to the library as NULL
            return None

    delete = torch.cuda.caching_allocator_delete

    def _free(ptr, nbytes, user):
        delete(ptr)

    a = vr_allocator()
    a.alloc = vr_allocator._fields_[0][1](_alloc)
    a.free = vr_allocator._fields_[1][1](_free)
    a.user = None
    a._keep = (_alloc, _free, a.alloc, a.free)
    return a


# contexts still open at interpreter exit are destroyed while PyTorch (which
# owns their device memory) is still intact
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for r in list(_LIVE):
        try:
            r.close()
        except Exception:  # noqa: BLE001
            pass


class Renderer:
    """One rendering context on a GPU (PyTorch tensors for outputs and streams)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, torch_alloc: bool = True):
        import torch
        self._torch = torch
        self.device = device
        self._alloc = torch_allocator(device) if (torch_alloc and device >= 0) else None
        h = P()
        check(lib().vr_create(device, budget_bytes,
                              ctypes.byref(self._alloc) if self._alloc else None, ctypes.byref(h)))
        self.ctx = h
        self._host_cubes = {}  # host arrays of registered cubes, alive until release
        _LIVE.add(self)

    def close(self):
        if self.ctx:
            check(lib().vr_destroy(self.ctx))
            self.ctx = None
            self._host_cubes = {}

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def _stream(self, stream):
        if stream is None:
            stream = self._torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    # -- cubes -----------------------------------------------------------------
    def upload(self, cube, storage="f32", sigma_scale=1.0, src_dtype=None, stream=None) -> int:
        """Upload a [nz][ny][nx] cube: a numpy array (float32, or uint16 codes with
        src_dtype 'f16'/'bf16') or a CUDA tensor of the same layout."""
        import numpy as np
        torch = self._torch
        on_dev = 0
        if isinstance(cube, torch.Tensor):
            arr = cube.contiguous()
            ptr = arr.data_ptr()
            on_dev = int(arr.is_cuda)
            dt = {torch.float32: VR_F32, torch.float16: VR_F16, torch.bfloat16: VR_BF16,
                  torch.int16: None, torch.uint16: None}.get(arr.dtype, "bad")
            if dt is None:
                dt = STORAGE[src_dtype]
            keep = arr
        else:
            arr = np.ascontiguousarray(cube)
            ptr = arr.ctypes.data
            if arr.dtype == np.float32:
                dt = VR_F32
            elif arr.dtype == np.uint16:
                dt = STORAGE[src_dtype]
            else:
                raise TypeError("cube must be float32 or uint16 codes")
            keep = arr
        if dt == "bad":
            raise TypeError("unsupported tensor dtype")
        nz, ny, nx = keep.shape
        out = ctypes.c_int32()
        check(lib().vr_cube_upload(self.ctx, ctypes.c_void_p(ptr), dt, on_dev, nx, ny, nz,
                                   STORAGE[storage], float(sigma_scale), self._stream(stream),
                                   ctypes.byref(out)))
        return out.value

    def register(self, cube, storage="f32", sigma_scale=1.0, src_dtype=None) -> int:
        """Register a host [nz][ny][nx] cube (numpy float32, or uint16 codes with
        src_dtype 'f16'/'bf16'; pinned torch CPU tensors also work) for on-demand
        admission under the context's memory budget.  The array is kept alive
        here until release."""
        import numpy as np
        torch = self._torch
        if isinstance(cube, torch.Tensor):
            if cube.is_cuda or not cube.is_contiguous():
                raise TypeError("register takes a contiguous host array")
            keep, ptr = cube, cube.data_ptr()
            dt = {torch.float32: VR_F32, torch.float16: VR_F16,
                  torch.bfloat16: VR_BF16}.get(cube.dtype)
            if dt is None:
                dt = STORAGE[src_dtype]
        else:
            keep = np.ascontiguousarray(cube)
            ptr = keep.ctypes.data
            if keep.dtype == np.float32:
                dt = VR_F32
            elif keep.dtype == np.uint16:
                dt = STORAGE[src_dtype]
            else:
                raise TypeError("cube must be float32 or uint16 codes")
        nz, ny, nx = keep.shape
        out = ctypes.c_int32()
        check(lib().vr_cube_register(self.ctx, ctypes.c_void_p(ptr), dt, nx, ny, nz,
                                     STORAGE[storage], float(sigma_scale), ctypes.byref(out)))
        self._host_cubes[out.value] = keep
        return out.value

    def _f32_source(self, cube):
        import numpy as np
        torch = self._torch
        if isinstance(cube, torch.Tensor):
            if cube.dtype != torch.float32:
                raise TypeError("float32 cube required")
            arr = cube.contiguous()
            return arr, arr.data_ptr(), int(arr.is_cuda)
        arr = np.ascontiguousarray(cube, dtype=np.float32)
        return arr, arr.ctypes.data, 0

    def estimate_channel_noise(self, cube, stream=None):
        """Per-channel (median, mad, sigma) of a float32 [nz][ny][nx] cube, as
        three numpy float32 arrays of nz values."""
        import numpy as np
        keep, ptr, on_dev = self._f32_source(cube)
        nz, ny, nx = keep.shape
        med, mad, sig = (np.empty(nz, np.float32) for _ in range(3))
        check(lib().vr_estimate_channel_noise(self.ctx, ctypes.c_void_p(ptr), on_dev, nx, ny, nz,
                                              self._stream(stream), med.ctypes.data,
                                              mad.ctypes.data, sig.ctypes.data))
        return med, mad, sig

    def upload_scaled(self, cube, divisors, storage="f32", stream=None) -> int:
        """Upload a float32 cube storing value / divisors[z] per channel."""
        import numpy as np
        keep, ptr, on_dev = self._f32_source(cube)
        nz, ny, nx = keep.shape
        d = np.ascontiguousarray(divisors, dtype=np.float32)
        if d.shape != (nz,):
            raise ValueError("one divisor per channel required")
        out = ctypes.c_int32()
        check(lib().vr_cube_upload_scaled(self.ctx, ctypes.c_void_p(ptr), on_dev, nx, ny, nz,
                                          STORAGE[storage], d.ctypes.data, self._stream(stream),
                                          ctypes.byref(out)))
        return out.value

    def memory_stats(self) -> dict:
        m = vr_memory_stats()
        check(lib().vr_get_memory_stats(self.ctx, ctypes.byref(m)))
        return m.as_dict()

    def release(self, cube: int):
        check(lib().vr_cube_release(self.ctx, cube))
        self._host_cubes.pop(cube, None)

    def info(self, cube: int) -> vr_cube_info:
        inf = vr_cube_info()
        check(lib().vr_cube_get_info(self.ctx, cube, ctypes.byref(inf)))
        return inf

    # -- state -----------------------------------------------------------------
    def set_transfer_function(self, rgbk, v0, v1):
        import numpy as np
        t = np.ascontiguousarray(np.asarray(rgbk, dtype=np.float32).reshape(-1, 4))
        check(lib().vr_set_transfer_function(self.ctx, t.ctypes.data, t.shape[0], v0, v1))

    def tf_create(self, rgbk, v0, v1) -> int:
        import numpy as np
        t = np.ascontiguousarray(np.asarray(rgbk, dtype=np.float32).reshape(-1, 4))
        out = ctypes.c_int32()
        check(lib().vr_tf_create(self.ctx, t.ctypes.data, t.shape[0], v0, v1, ctypes.byref(out)))
        return out.value

    def tf_release(self, tf: int):
        check(lib().vr_tf_release(self.ctx, tf))

    def set_noise_clip(self, k, sigma=1.0):
        check(lib().vr_set_noise_clip(self.ctx, k, sigma))

    def set_camera(self, cam):
        c = make_camera(cam)
        check(lib().vr_set_camera(self.ctx, ctypes.byref(c)))

    # -- rendering -------------------------------------------------------------
    def output(self, width, height, mode="ea"):
        torch = self._torch
        shape = (height, width, 4) if mode in ("ea", VR_EA) else (height, width)
        return torch.empty(shape, dtype=torch.float32, device="cuda:%d" % self.device)

    def render(self, cube, width, height, mode="ea", interp="trilinear", step=0.5, ert=0.99,
               use_skip=True, out=None, stream=None, stats=False):
        p = make_params(width, height, mode, interp, step, ert, use_skip)
        if out is None:
            out = self.output(width, height, mode)
        st = vr_stats() if stats else None
        check(lib().vr_render(self.ctx, cube, ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                              self._stream(stream), ctypes.byref(st) if st is not None else None))
        return (out, st.as_dict()) if stats else out

    def render_subcube(self, cube, width, height, axis, plane_lo, plane_hi, mode="ea",
                       interp="trilinear", step=0.5, ert=0.99, use_skip=True, out=None,
                       stream=None, stats=False):
        """Partial image of the sub-cube of planes [plane_lo, plane_hi) on `axis`."""
        p = make_params(width, height, mode, interp, step, ert, use_skip)
        if out is None:
            out = self.output(width, height, mode)
        st = vr_stats() if stats else None
        check(lib().vr_render_subcube(self.ctx, cube, ctypes.byref(p), int(axis), int(plane_lo),
                                      int(plane_hi), ctypes.c_void_p(out.data_ptr()),
                                      self._stream(stream),
                                      ctypes.byref(st) if st is not None else None))
        return (out, st.as_dict()) if stats else out

    def composite(self, partials, axis, width, height, mode="ea", out=None, stream=None):
        """Integrate partial images (sub-cubes in increasing plane order)."""
        if out is None:
            out = self.output(width, height, mode)
        arr = (ctypes.c_void_p * len(partials))(*[t.data_ptr() for t in partials])
        m = {"ea": VR_EA, "mip": VR_MIP}[mode] if isinstance(mode, str) else int(mode)
        check(lib().vr_composite(self.ctx, m, arr, len(partials), int(axis), int(width),
                                 int(height), ctypes.c_void_p(out.data_ptr()), self._stream(stream)))
        return out

    def render_progressive(self, cube, width, height, out, budget_ms, max_level=3, mode="ea",
                           interp="trilinear", step=0.5, ert=0.99, use_skip=True, stream=None):
        """One call of the coarse-to-fine loop (see vr_render_progressive); returns
        its info as a dict."""
        p = make_params(width, height, mode, interp, step, ert, use_skip)
        info = vr_progressive_info()
        check(lib().vr_render_progressive(self.ctx, cube, ctypes.byref(p), float(budget_ms),
                                          int(max_level), ctypes.c_void_p(out.data_ptr()),
                                          self._stream(stream), ctypes.byref(info)))
        return info.as_dict()

    def request(self, cube, cam, width, height, out, mode="ea", interp="trilinear", step=0.5,
                ert=0.99, use_skip=True, tf=0, clip=-math.inf) -> vr_request:
        r = vr_request()
        r.cube = cube
        r.tf = tf
        r.clip = clip
        r.camera = make_camera(cam)
        r.params = make_params(width, height, mode, interp, step, ert, use_skip)
        r.out_dev = out.data_ptr()
        return r

    def render_batch(self, requests, stream=None, stats=False):
        n = len(requests)
        arr = (vr_request * n)(*requests)
        st = (vr_stats * n)() if stats else None
        check(lib().vr_render_batch(self.ctx, arr, n, self._stream(stream), st))
        return [s.as_dict() for s in st] if stats else None

    # -- serving ---------------------------------------------------------------
    def server_start(self, max_batch_requests=64, max_batch_tiles=16384, max_inflight=2,
                     use_graphs=1):
        cfg = vr_server_cfg(max_batch_requests, max_batch_tiles, max_inflight, use_graphs)
        check(lib().vr_server_start(self.ctx, ctypes.byref(cfg)))

    def server_stop(self):
        check(lib().vr_server_stop(self.ctx))

    def submit(self, request: vr_request) -> int:
        t = ctypes.c_uint64()
        check(lib().vr_submit(self.ctx, ctypes.byref(request), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        check(lib().vr_poll(self.ctx, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_s: float = 0.0) -> float:
        lat = ctypes.c_double()
        check(lib().vr_wait(self.ctx, ticket, timeout_s, ctypes.byref(lat)))
        return lat.value
