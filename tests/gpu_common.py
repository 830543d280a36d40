"""Shared helpers for the GPU tests: renderer fixture plumbing and comparisons
against the FP64 reference with its ambiguity flags."""
import math

import numpy as np

import oracle

# Per-channel absolute tolerance for float32 storage (RGBA in [0, 1]) and the
# relative tolerance for MIP values, max(1, |m|)-scaled.
TOL_F32 = 1e-5
# Float16/bfloat16 storage, measured against the reference on the original float32 cube.
TOL_16 = 4e-3


def ref_render(vol, wl_kw, camera, W, H, mode, interp, pixels=None, **extra):
    kw = dict(wl_kw)
    kw.update(extra)
    return oracle.render(vol, mode=oracle.MIP if mode == "mip" else oracle.EA,
                         interp=oracle.NEAREST if interp == "nearest" else oracle.TRILINEAR,
                         camera=camera, width=W, height=H, pixels=pixels, **kw)


def compare_ea(gpu, ref, tol, flags=None, max_ambiguous_frac=0.01):
    """gpu: (..., 4) float32; ref: (..., 4) float64 with matching flags.
    Strict tolerance on unambiguous pixels; ambiguous ones (several correct
    results) are counted and bounded by the early-termination remainder."""
    gpu = np.asarray(gpu, dtype=np.float64)
    err = np.abs(gpu - ref).max(axis=-1)
    if flags is None:
        amb = np.zeros(err.shape, dtype=bool)
    else:
        amb = (flags & oracle.FLAGS_AMBIGUOUS) > 0
    strict = err[~amb]
    worst = float(strict.max()) if strict.size else 0.0
    rms = float(np.sqrt(np.mean(strict ** 2))) if strict.size else 0.0
    info = {"max_err": worst, "rms_err": rms, "n_ambiguous": int(amb.sum()), "n": int(err.size)}
    assert worst <= tol, info
    if amb.any():
        assert amb.mean() <= max_ambiguous_frac, info
        assert float(err[amb].max()) <= 0.01 + tol, info
    return info


def compare_mip(gpu, ref, tol, flags=None):
    gpu = np.asarray(gpu, dtype=np.float64)
    miss_g, miss_r = np.isneginf(gpu), np.isneginf(ref)
    amb = np.zeros(gpu.shape, dtype=bool) if flags is None else (flags & oracle.FLAGS_AMBIGUOUS) > 0
    assert np.array_equal(miss_g[~amb], miss_r[~amb]), "hit/miss pattern differs"
    hit = ~miss_r & ~miss_g & ~amb
    err = np.abs(gpu[hit] - ref[hit]) / np.maximum(1.0, np.abs(ref[hit]))
    worst = float(err.max()) if err.size else 0.0
    info = {"max_rel_err": worst, "n_ambiguous": int(amb.sum()), "n": int(gpu.size)}
    assert worst <= tol, info
    return info


def wl_kwargs(wl, tf):
    """Reference keyword arguments for a workload (float32 TF rows promoted exactly)."""
    return dict(tf=np.asarray(tf, dtype=np.float64), v0=wl.v0, v1=wl.v1,
                clip=wl.clip_k * wl.cube.sigma, step=wl.step, ert=float(np.float32(wl.ert)))


def set_state(r, wl, tf, camera, clip=True):
    r.set_transfer_function(tf, wl.v0, wl.v1)
    r.set_noise_clip(wl.clip_k if clip else -math.inf, wl.cube.sigma)
    r.set_camera(camera)
