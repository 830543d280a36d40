"""Seeded synthetic inputs shared by the renderer's tests/benchmarks and the CPU reference.

This module produces *inputs only*: voxel values of noisy spectral cubes,
transfer-function tables, camera poses and pixel subsets.  It holds none of
the rendering arithmetic (no ray set-up, sampling, classification or
compositing), so the GPU path and the CPU reference stay independent while
consuming identical bytes.

The cube model follows Sec. 2 of the paper (two sky axes plus one frequency
axis, stored as a stack of channel images, x fastest).  Workload recipes
(sizes, source populations, seeds) are the configurations the renderer is
benchmarked and checked on.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so (plain C, gcc)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, dbl, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.synth_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.synth_philox4x32_10.restype = None
        L.synth_normal.argtypes = [u64, u64]
        L.synth_normal.restype = dbl
        L.synth_uniforms.argtypes = [u64, u64, i64, ctypes.c_void_p]
        L.synth_uniforms.restype = None
        L.synth_sources.argtypes = [u64, i64, i64, i64, i64, dbl, dbl, i32, dbl, dbl, dbl, dbl,
                                    ctypes.c_void_p]
        L.synth_sources.restype = i32
        L.synth_cube.argtypes = [u64, i64, i64, i64, dbl, ctypes.c_void_p, i64, i32, i64, i64,
                                 ctypes.c_void_p, i32]
        L.synth_cube.restype = i32
        _lib = L
    return _lib


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def philox4x32_10(ctr, key):
    """The raw Philox4x32-10 bijection (4 counter words, 2 key words) -> 4 words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().synth_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def normal(seed: int, index: int) -> float:
    return float(lib().synth_normal(seed, index))


def uniforms(seed: int, index: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    lib().synth_uniforms(seed, index, count, out.ctypes.data)
    return out


# ----------------------------------------------------------------------------
# Cubes
# ----------------------------------------------------------------------------
@dataclass
class SourcePop:
    """Population of 3-D Gaussian sources (amplitudes in units of sigma)."""
    count: int
    a_lo: float
    a_hi: float
    a_log: bool
    ss_lo: float
    ss_hi: float
    sz_lo: float
    sz_hi: float


@dataclass
class CubeSpec:
    nx: int
    ny: int
    nz: int
    seed: int
    sources: SourcePop | None = None
    sigma: float = 1.0
    noise: bool = True

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nbytes_f32(self) -> int:
        return 4 * self.nx * self.ny * self.nz


def source_catalogue(spec: CubeSpec) -> np.ndarray:
    p = spec.sources
    if p is None or p.count == 0:
        return np.zeros((0, 6), dtype=np.float64)
    out = np.empty((p.count, 6), dtype=np.float64)
    rc = lib().synth_sources(spec.seed, p.count, spec.nx, spec.ny, spec.nz, p.a_lo, p.a_hi,
                             int(p.a_log), p.ss_lo, p.ss_hi, p.sz_lo, p.sz_hi, out.ctypes.data)
    if rc != 0:
        raise ValueError("synth_sources failed")
    return out


def cube_slab(spec: CubeSpec, z0: int, nzs: int, src: np.ndarray | None = None,
              threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Float32 planes z0..z0+nzs-1 of the cube, shape (nzs, ny, nx)."""
    if src is None:
        src = source_catalogue(spec)
    src = np.ascontiguousarray(src, dtype=np.float64)
    if out is None:
        out = np.empty((nzs, spec.ny, spec.nx), dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.shape == (nzs, spec.ny, spec.nx)
    rc = lib().synth_cube(spec.seed, spec.nx, spec.ny, spec.nz, spec.sigma,
                          src.ctypes.data if len(src) else None, len(src), int(spec.noise), z0, nzs,
                          out.ctypes.data, threads or default_threads())
    if rc != 0:
        raise RuntimeError("synth_cube failed (%d)" % rc)
    return out


def cube(spec: CubeSpec, threads: int | None = None) -> np.ndarray:
    """The whole cube as float32 [nz][ny][nx]."""
    return cube_slab(spec, 0, spec.nz, threads=threads)


# ----------------------------------------------------------------------------
# Transfer functions (tables are inputs)
# ----------------------------------------------------------------------------
def ramp_tf(n: int = 256, kappa_max: float = 1.0) -> np.ndarray:
    """Linear RGBA ramp with distinct channels: row i = (s, s/2, 1-s, kappa_max*s), s=i/(n-1).

    The fourth channel is an extinction coefficient per voxel length.
    """
    s = np.arange(n, dtype=np.float64) / (n - 1)
    return np.stack([s, 0.5 * s, 1.0 - s, kappa_max * s], axis=1).astype(np.float32)


# ----------------------------------------------------------------------------
# Cameras (poses are inputs)
# ----------------------------------------------------------------------------
@dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple
    fovy_deg: float = 60.0
    ortho: bool = False
    ortho_w: float = 0.0
    ortho_h: float = 0.0


def box_centre(nx, ny, nz):
    return ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)


def bounding_radius(nx, ny, nz):
    """Radius of the sphere around the cell-centred box [-1/2, N-1/2]^3."""
    return 0.5 * math.sqrt(nx * nx + ny * ny + nz * nz)


def orbit_camera(nx, ny, nz, theta, phi, fovy_deg=60.0, dist_factor=2.0) -> Camera:
    """Perspective camera on a sphere of radius dist_factor*r_b around the box centre.

    With dist_factor 2 and a 60 degree field of view the bounding sphere exactly
    fills the image height.  Up is +z unless the view is nearly polar.
    """
    c = box_centre(nx, ny, nz)
    R = dist_factor * bounding_radius(nx, ny, nz)
    e = (c[0] + R * math.cos(phi) * math.cos(theta), c[1] + R * math.cos(phi) * math.sin(theta),
         c[2] + R * math.sin(phi))
    up = (0.0, 1.0, 0.0) if abs(math.sin(phi)) > 0.99 else (0.0, 0.0, 1.0)
    return Camera(eye=e, target=c, up=up, fovy_deg=fovy_deg)


def orbit_angles(seed: int, count: int, phi_max_deg: float = 45.0):
    """Seeded orbit angles: theta ~ U[0, 2 pi), phi ~ U[-phi_max, phi_max]."""
    out = []
    for i in range(count):
        u = uniforms(seed, i, 2)
        out.append((2.0 * math.pi * u[0], math.radians(phi_max_deg) * (2.0 * u[1] - 1.0)))
    return out


def axis_camera(nx, ny, nz, axis: str, W: int, H: int) -> Camera:
    """Orthographic axis-aligned view of the whole box, letterboxed to W x H.

    axis 'z': looks along +z, image columns follow +x, rows follow +y.
    axis 'x': looks along +x, columns follow +y, rows follow +z.
    axis 'y': looks along -y, columns follow +x, rows follow +z.
    """
    c = box_centre(nx, ny, nz)
    if axis == "z":
        f, up, ext = (0, 0, 1), (0, -1, 0), (nx, ny)
    elif axis == "x":
        f, up, ext = (1, 0, 0), (0, 0, -1), (ny, nz)
    elif axis == "y":
        f, up, ext = (0, -1, 0), (0, 0, -1), (nx, nz)
    else:
        raise ValueError(axis)
    # window covering the box face, same aspect as the image
    w, h = float(ext[0]), float(ext[1])
    if w / h > W / H:
        h = w * H / W
    else:
        w = h * W / H
    eye = (c[0] - f[0], c[1] - f[1], c[2] - f[2])
    return Camera(eye=eye, target=c, up=up, ortho=True, ortho_w=w, ortho_h=h)


def pixel_subset(seed: int, W: int, H: int, count: int) -> np.ndarray:
    """Seeded distinct pixel coordinates as int32 (count, 2) rows of (i=column, j=row)."""
    count = min(count, W * H)
    u = uniforms(seed, 0x7FFFFFFF, 2 * count + 64)
    picked = np.unique((u * (W * H)).astype(np.int64) % (W * H))[:count]
    k = 1
    while len(picked) < count:
        extra = (uniforms(seed, 0x7FFFFFFF + k, count) * (W * H)).astype(np.int64)
        picked = np.unique(np.concatenate([picked, extra]))[:count]
        k += 1
    return np.stack([picked % W, picked // W], axis=1).astype(np.int32)


# ----------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    cube: CubeSpec
    width: int
    height: int
    v0: float
    v1: float
    clip_k: float
    kappa_max: float = 1.0
    step: float = 0.5
    ert: float = 0.99
    extra: dict = field(default_factory=dict)


def tiny() -> Workload:
    """64x64x128 float32 cube: noise plus 3 sources (peak 5-20 sigma, widths 2-6 voxels);
    orthographic axis-aligned 256x256 views, ramp TF over [3, 20] sigma clipped below 3 sigma."""
    spec = CubeSpec(64, 64, 128, seed=1001,
                    sources=SourcePop(3, 5.0, 20.0, False, 2.0, 6.0, 2.0, 6.0))
    return Workload("tiny-64x64x128", spec, 256, 256, v0=3.0, v1=20.0, clip_k=3.0)


def full() -> Workload:
    """512x512x1024 float32 cube: noise plus 200 sources (peaks log-uniform 3-50 sigma,
    spatial widths 1-8, spectral widths 2-40 channels); 1024x1024 perspective orbit views,
    ramp TF over [3, 50] sigma clipped below 3 sigma, step 0.5, early termination at 0.99."""
    spec = CubeSpec(512, 512, 1024, seed=1002,
                    sources=SourcePop(200, 3.0, 50.0, True, 1.0, 8.0, 2.0, 40.0))
    return Workload("full-512x512x1024", spec, 1024, 1024, v0=3.0, v1=50.0, clip_k=3.0,
                    extra={"camera_seed": 2002, "n_views": 16})


def large() -> Workload:
    """2048x2048x4096 cube (stored FP16): noise plus 5000 sources, 2048x2048 perspective,
    ramp over [4, 50] sigma clipped below 4 sigma."""
    spec = CubeSpec(2048, 2048, 4096, seed=1005,
                    sources=SourcePop(5000, 3.0, 50.0, True, 1.0, 8.0, 2.0, 40.0))
    return Workload("large-2048x2048x4096", spec, 2048, 2048, v0=4.0, v1=50.0, clip_k=4.0,
                    extra={"camera_seed": 2005})


def serving_cubes(count: int = 8, base_seed: int = 10040):
    """Cubes for the serving workload: Nx, Ny ~ U{128..1024}, Nz ~ U{128..512};
    source count density-matched to the full-size workload."""
    specs = []
    for i in range(count):
        u = uniforms(base_seed + i, 0, 3)
        nx = 128 + int(u[0] * (1024 - 128 + 1))
        ny = 128 + int(u[1] * (1024 - 128 + 1))
        nz = 128 + int(u[2] * (512 - 128 + 1))
        ns = max(1, int(round(200.0 * nx * ny * nz / (512.0 * 512.0 * 1024.0))))
        specs.append(CubeSpec(nx, ny, nz, seed=base_seed + i,
                              sources=SourcePop(ns, 3.0, 50.0, True, 1.0, 8.0, 2.0, 40.0)))
    return specs
