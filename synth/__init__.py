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


def band_noise_profile(nz: int) -> np.ndarray:
    """Noise level per frequency channel for the noise-aware workloads: rising
    towards the upper band edge (1 -> 1.6) with a narrow interference bump
    (+0.8 at 30 % of the band, width 5 % of the band)."""
    z = np.arange(nz, dtype=np.float64)
    t = z / max(nz - 1, 1)
    return 1.0 + 0.6 * t * t + 0.8 * np.exp(-((z - 0.3 * nz) / (0.05 * nz)) ** 2)


def cube_profiled(spec: CubeSpec, profile: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Cube whose noise level varies per channel: profile[z] times the unit
    noise of `spec` plus its sources, rounded once to float32."""
    import dataclasses
    prof = np.asarray(profile, dtype=np.float64)
    assert prof.shape == (spec.nz,)
    noise = cube(dataclasses.replace(spec, sources=None, sigma=1.0, noise=True), threads)
    srcs = cube(dataclasses.replace(spec, noise=False), threads)
    return (prof[:, None, None] * noise.astype(np.float64) + srcs.astype(np.float64)).astype(np.float32)


# ----------------------------------------------------------------------------
# The same generator evaluated on the GPU (for cubes too large to generate on
# the host in reasonable time).  Source factors are tabulated here with the C
# library's exp, in the operation order of synth.c, so source terms match the
# CPU generator bit for bit; see synth_gpu.hip for the noise.
# ----------------------------------------------------------------------------
_GPU_SRC = os.path.join(_HERE, "synth_gpu.hip")
_GPU_LIB_PATH = os.path.join(_HERE, "libsynth_gpu.so")
_gpu_lib = None


def build_gpu(force: bool = True) -> str:
    """Compile synth_gpu.hip into libsynth_gpu.so (hipcc, gfx950)."""
    if force or not os.path.exists(_GPU_LIB_PATH):
        tmp = _GPU_LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, _GPU_SRC])
        os.replace(tmp, _GPU_LIB_PATH)
    return _GPU_LIB_PATH


def gpu_lib():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_LIB_PATH):
            raise RuntimeError("libsynth_gpu.so is not built (synth.build_gpu())")
        # PyTorch's HIP runtime must be the one in the process before this
        # library resolves its own runtime dependency to the same soname
        import torch  # noqa: F401
        L = ctypes.CDLL(_GPU_LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.synth_gpu_planes.argtypes = [ctypes.c_uint64, i64, i64, ctypes.c_double, ctypes.c_int, i64, i64,
                                       vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
        L.synth_gpu_planes.restype = ctypes.c_int
        _gpu_lib = L
    return _gpu_lib


def source_tables(spec: CubeSpec, src: np.ndarray):
    """Per-source rectangles and x / y factor tables, as synth.c evaluates them."""
    nx, ny = spec.nx, spec.ny
    rect = np.zeros((len(src), 4), dtype=np.int32)
    fx_off = np.zeros(len(src), dtype=np.int64)
    fy_off = np.zeros(len(src), dtype=np.int64)
    fx, fy, live = [], [], np.zeros(len(src), dtype=bool)
    for s, (x0, y0, zc, A, ss, sz) in enumerate(src.tolist()):
        xa = max(int(math.ceil(x0 - 5.0 * ss)), 0)
        xb = min(int(math.floor(x0 + 5.0 * ss)), nx - 1)
        ya = max(int(math.ceil(y0 - 5.0 * ss)), 0)
        yb = min(int(math.floor(y0 + 5.0 * ss)), ny - 1)
        if xa > xb or ya > yb:
            continue
        live[s] = True
        rect[s] = (xa, xb, ya, yb)
        fx_off[s] = len(fx)
        for x in range(xa, xb + 1):
            dx = float(x) - x0
            fx.append(math.exp(-0.5 * dx * dx / (ss * ss)))
        fy_off[s] = len(fy)
        for y in range(ya, yb + 1):
            dy = float(y) - y0
            fy.append(math.exp(-0.5 * dy * dy / (ss * ss)))
    return rect, fx_off, fy_off, np.asarray(fx or [0.0]), np.asarray(fy or [0.0]), live


def plane_entries(spec: CubeSpec, src: np.ndarray, live: np.ndarray, z0: int, nzs: int):
    """For planes z0 .. z0+nzs-1: CSR offsets, source indices (catalogue order)
    and factors A * sigma * exp(-dz^2 / (2 sz^2)) of the sources that reach them."""
    zs, ss_, aa = [], [], []
    for s, (x0, y0, zc, A, ssp, sz) in enumerate(src.tolist()):
        if not live[s]:
            continue
        lo = max(int(math.floor(zc - 5.0 * sz)) - 1, z0)
        hi = min(int(math.ceil(zc + 5.0 * sz)) + 1, z0 + nzs - 1)
        for z in range(lo, hi + 1):
            dz = float(z) - zc
            if abs(dz) > 5.0 * sz:
                continue
            zs.append(z - z0)
            ss_.append(s)
            aa.append(A * spec.sigma * math.exp(-0.5 * dz * dz / (sz * sz)))
    zs = np.asarray(zs, dtype=np.int64)
    ss_ = np.asarray(ss_, dtype=np.int32)
    aa = np.asarray(aa, dtype=np.float64)
    order = np.lexsort((ss_, zs))
    zs, ss_, aa = zs[order], ss_[order], aa[order]
    off = np.zeros(nzs + 1, dtype=np.int64)
    np.add.at(off, zs + 1, 1)
    off = np.cumsum(off)
    return off, (ss_ if len(ss_) else np.zeros(1, np.int32)), (aa if len(aa) else np.zeros(1))


def cube_gpu(spec: CubeSpec, out, chunk: int = 64) -> None:
    """Fill `out` (a contiguous float32 CUDA tensor of shape (nz, ny, nx)) with the cube."""
    import torch
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
    assert tuple(out.shape) == (spec.nz, spec.ny, spec.nx)
    dev = out.device
    src = source_catalogue(spec)
    rect, fx_off, fy_off, fx, fy, live = source_tables(spec, src)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d_rect, d_fxo, d_fyo, d_fx, d_fy = t(rect.reshape(-1) if len(rect) else np.zeros(4, np.int32)), \
        t(fx_off if len(fx_off) else np.zeros(1, np.int64)), t(fy_off if len(fy_off) else np.zeros(1, np.int64)), t(fx), t(fy)
    stream = torch.cuda.current_stream(dev).cuda_stream
    for z0 in range(0, spec.nz, chunk):
        nzs = min(chunk, spec.nz - z0)
        off, ents, aa = plane_entries(spec, src, live, z0, nzs)
        d_off, d_ent, d_a = t(off), t(ents), t(aa)
        rc = gpu_lib().synth_gpu_planes(spec.seed, spec.nx, spec.ny, spec.sigma, int(spec.noise), z0, nzs,
                                        d_off.data_ptr(), d_ent.data_ptr(), d_a.data_ptr(),
                                        d_rect.data_ptr(), d_fxo.data_ptr(), d_fyo.data_ptr(),
                                        d_fx.data_ptr(), d_fy.data_ptr(), out[z0].data_ptr(),
                                        dev.index if dev.index is not None else 0, stream)
        if rc != 0:
            raise RuntimeError("synth_gpu_planes failed (%d)" % rc)
    torch.cuda.synchronize(dev)


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
