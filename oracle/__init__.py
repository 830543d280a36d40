"""FP64 CPU reference ray caster — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The renderer itself never calls it and shares no code
with it.  See ``vr_oracle.c`` for what is computed and which passages of the
paper it follows (Sec. 2, design decision 1: ray-casting volume rendering;
Sec. 3, process step 3: each pixel mapped to RGBA by a pre-selected transfer
function).

Besides the C ray caster this module holds the reference conversions of float32
voxels to the 16-bit storage formats (round to nearest even), used to build the
reference's inputs for the reduced-precision storage form.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

F32, F16, BF16, F64 = 0, 1, 2, 3
EA, MIP = 0, 1
NEAREST, TRILINEAR = 0, 1

FLAG_HIT = 1
FLAG_ERT_AMBIG = 2
FLAG_CLIP_AMBIG = 4
FLAG_NEAREST_AMBIG = 8
FLAG_GRAZE_AMBIG = 16
FLAG_MIPCLIP_AMBIG = 32
FLAG_ERT_STOPPED = 64
FLAG_WINDOW_AMBIG = 128
FLAGS_AMBIGUOUS = (FLAG_ERT_AMBIG | FLAG_CLIP_AMBIG | FLAG_NEAREST_AMBIG | FLAG_GRAZE_AMBIG
                   | FLAG_MIPCLIP_AMBIG | FLAG_WINDOW_AMBIG)
# MIP partial of a sub-cube whose samples all lie below the clip
MIP_BELOW_CLIP = -3.4028234663852886e38


def build(force: bool = True) -> str:
    """Compile vr_oracle.c (plain C99, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Scene(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("vox", ctypes.c_void_p), ("vox_dtype", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("vox_scale", ctypes.c_double),
        ("tf", ctypes.c_void_p), ("tf_n", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("v0", ctypes.c_double), ("v1", ctypes.c_double), ("clip", ctypes.c_double),
        ("interp", ctypes.c_int32), ("ortho", ctypes.c_int32),
        ("step", ctypes.c_double), ("ert", ctypes.c_double),
        ("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
        ("fovy_deg", ctypes.c_double), ("ortho_w", ctypes.c_double), ("ortho_h", ctypes.c_double),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("amb_ert", ctypes.c_double), ("amb_clip", ctypes.c_double),
        ("amb_nearest", ctypes.c_double), ("amb_graze", ctypes.c_double),
        ("win_axis", ctypes.c_int32), ("pad1", ctypes.c_int32),
        ("win_lo", ctypes.c_double), ("win_hi", ctypes.c_double), ("amb_window", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_render.argtypes = [ctypes.POINTER(Scene), ctypes.c_int64, P, P, P, P, P, P,
                                 ctypes.c_int]
        L.orc_render.restype = ctypes.c_int
        L.orc_decode_f16.argtypes = [ctypes.c_uint16]
        L.orc_decode_f16.restype = ctypes.c_double
        L.orc_decode_bf16.argtypes = [ctypes.c_uint16]
        L.orc_decode_bf16.restype = ctypes.c_double
        L.orc_pixel_ray.argtypes = [ctypes.POINTER(Scene), ctypes.c_int64, ctypes.c_int64, P, P]
        L.orc_pixel_ray.restype = None
        L.orc_slab.argtypes = [ctypes.POINTER(Scene), P, P, P, P]
        L.orc_slab.restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


# ----------------------------------------------------------------------------
# Reference storage conversions (round to nearest, ties to even)
# ----------------------------------------------------------------------------
def to_f16_bits(x: np.ndarray) -> np.ndarray:
    """IEEE binary16 bits of x (float32), round to nearest even (numpy's cast)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """bfloat16 bits of x (float32): the upper 16 bits after round-to-nearest-even."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def decode_bits(bits: np.ndarray, dtype: int) -> np.ndarray:
    """Exact float64 values of 16-bit storage codes."""
    b = np.asarray(bits, dtype=np.uint16)
    if dtype == F16:
        return b.view(np.float16).astype(np.float64)
    if dtype == BF16:
        return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    raise ValueError(dtype)


# ----------------------------------------------------------------------------
# Rendering
# ----------------------------------------------------------------------------
def make_scene(vol, *, mode=EA, interp=TRILINEAR, tf=None, v0=0.0, v1=1.0, clip=-math.inf,
               step=0.5, ert=0.99, camera=None, width=1, height=1, vox_dtype=None, vox_scale=1.0,
               amb_ert=1e-5, amb_clip=1e-4, amb_nearest=1e-6, amb_graze=1e-6, window=None,
               amb_window=1e-6):
    """Build the scene struct.  ``vol`` is [nz][ny][nx] float32/float64, or uint16
    storage codes with ``vox_dtype`` F16/BF16.  Keeps references alive on the struct."""
    vol = np.ascontiguousarray(vol)
    if vox_dtype is None:
        vox_dtype = {np.dtype(np.float32): F32, np.dtype(np.float64): F64}[vol.dtype]
    if vox_dtype in (F16, BF16):
        assert vol.dtype == np.uint16
    nz, ny, nx = vol.shape
    S = Scene()
    S.nx, S.ny, S.nz = nx, ny, nz
    S.vox = vol.ctypes.data
    S.vox_dtype = vox_dtype
    S.vox_scale = vox_scale
    if tf is not None:
        tfa = np.ascontiguousarray(np.asarray(tf, dtype=np.float64).reshape(-1, 4))
        S.tf = tfa.ctypes.data
        S.tf_n = tfa.shape[0]
    else:
        tfa = None
        S.tf = None
        S.tf_n = 0
    S.mode, S.interp = mode, interp
    S.v0, S.v1, S.clip = v0, v1, clip
    S.step, S.ert = step, ert
    cam = camera
    S.ortho = int(bool(cam.ortho))
    for a in range(3):
        S.eye[a], S.target[a], S.up[a] = cam.eye[a], cam.target[a], cam.up[a]
    S.fovy_deg, S.ortho_w, S.ortho_h = cam.fovy_deg, cam.ortho_w, cam.ortho_h
    S.width, S.height = width, height
    S.amb_ert, S.amb_clip, S.amb_nearest, S.amb_graze = amb_ert, amb_clip, amb_nearest, amb_graze
    # sub-cube window (axis, lo, hi): only samples with lo <= p[axis] < hi
    if window is None:
        S.win_axis, S.win_lo, S.win_hi = -1, -math.inf, math.inf
    else:
        S.win_axis, S.win_lo, S.win_hi = int(window[0]), float(window[1]), float(window[2])
    S.amb_window = amb_window
    S._keep = (vol, tfa)
    return S


def render(vol, *, pixels=None, threads=None, **kw):
    """Render the full image (pixels=None) or a list of (i, j) pixels.

    Returns a dict with ``image`` (H, W, 4) / (H, W) for full images or
    ``values`` (npix, 4) / (npix,) for pixel lists, plus ``n_nominal``,
    ``n_exec`` and ``flags`` with matching leading shape; for MIP also
    ``bounds`` (..., 2): the least and greatest correct maximum where nearest
    sampling meets rounding ties (equal to the value elsewhere).
    """
    S = make_scene(vol, **kw)
    W, H = S.width, S.height
    ch = 1 if S.mode == MIP else 4
    if pixels is None:
        npix = W * H
        px = None
    else:
        px = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
        npix = px.shape[0]
    out = np.zeros((npix, ch), dtype=np.float64)
    nn = np.zeros(npix, dtype=np.int64)
    ne = np.zeros(npix, dtype=np.int64)
    fl = np.zeros(npix, dtype=np.int32)
    bd = np.zeros((npix, 2), dtype=np.float64) if ch == 1 else None
    rc = lib().orc_render(ctypes.byref(S), npix, px.ctypes.data if px is not None else None,
                          out.ctypes.data, nn.ctypes.data, ne.ctypes.data, fl.ctypes.data,
                          bd.ctypes.data if bd is not None else None,
                          threads or default_threads())
    if rc != 0:
        raise ValueError("orc_render rejected its arguments")
    if ch == 1:
        out = out[:, 0]
    res = {"n_nominal": nn, "n_exec": ne, "flags": fl}
    if bd is not None:
        res["bounds"] = bd
    if pixels is None:
        res["image"] = out.reshape((H, W, 4) if ch == 4 else (H, W))
        res["n_nominal"] = nn.reshape(H, W)
        res["n_exec"] = ne.reshape(H, W)
        res["flags"] = fl.reshape(H, W)
        if bd is not None:
            res["bounds"] = bd.reshape(H, W, 2)
    else:
        res["values"] = out
    return res


def composite_over(partials):
    """Front-to-back "over" of premultiplied RGBA partial images (..., 4), the
    first in front: C = C_f + (1 - A_f) C_b, A = A_f + (1 - A_f) A_b (Porter and
    Duff 1984); the scene integration of sub-cube images (Sec. 3.1, step 5)."""
    acc = np.zeros_like(np.asarray(partials[0], dtype=np.float64))
    for p in partials:
        p = np.asarray(p, dtype=np.float64)
        acc = acc + (1.0 - acc[..., 3:4]) * p
    return acc


def composite_max(partials):
    """MIP partials combined by maximum, then the clip floor: -inf where no
    sub-cube held a sample, 0 where all samples lay below the clip."""
    m = np.max(np.stack([np.asarray(p, dtype=np.float64) for p in partials]), axis=0)
    return np.where(m == MIP_BELOW_CLIP, 0.0, m)


def pixel_ray(camera, width, height, i, j):
    """The reference's ray (origin, unit direction) for pixel (i, j)."""
    dummy = np.zeros((2, 2, 2), dtype=np.float32)
    S = make_scene(dummy, camera=camera, width=width, height=height, mode=MIP)
    o = np.zeros(3)
    d = np.zeros(3)
    lib().orc_pixel_ray(ctypes.byref(S), i, j, o.ctypes.data, d.ctypes.data)
    return o, d


def slab(shape_zyx, camera, width, height, o, d):
    """The reference's slab test: (hit, t_in, t_out)."""
    nz, ny, nx = shape_zyx
    dummy = np.zeros((2, 2, 2), dtype=np.float32)
    S = make_scene(dummy, camera=camera, width=width, height=height, mode=MIP)
    S.nx, S.ny, S.nz = nx, ny, nz
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    ti = ctypes.c_double()
    to = ctypes.c_double()
    hit = lib().orc_slab(ctypes.byref(S), o.ctypes.data, d.ctypes.data, ctypes.byref(ti),
                         ctypes.byref(to))
    return bool(hit), ti.value, to.value
