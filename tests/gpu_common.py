"""Shared helpers for the GPU tests: renderer fixture plumbing and comparisons
against the FP64 reference with its ambiguity flags."""
import json
import math
import os

import numpy as np

import oracle

# Per-channel absolute tolerance for float32 storage (RGBA in [0, 1]) and the
# relative tolerance for MIP values, max(1, |m|)-scaled.
TOL_F32 = 1e-5
# Float16/bfloat16 storage, measured against the reference on the original float32 cube.
TOL_16 = 4e-3


def ref_render(vol, wl_kw, camera, W, H, mode, interp, pixels=None, **extra):
    """The FP64 reference for one image or pixel list (see oracle.render)."""
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


def compare_mip(gpu, ref, tol, flags=None, bounds=None, clip=-math.inf, max_loose_frac=0.01,
                amb_clip=1e-4):
    """gpu: float32 MIP values; ref: float64 reference values (-inf = miss),
    with the reference's flags and, for nearest sampling, its bounds of the
    correct maxima (..., 2).  Tolerance: tol * max(1, |m|) (MIP values are in
    data units, and float32 arithmetic on a value m rounds at about |m| * 2^-24
    per operation); the absolute error is reported beside it.

    Pixels where several results are correct are each checked against their
    own set of correct results:
      * nearest-sampling tie: the value is x (or 0 when x < clip) for some x
        in [lo, hi], the least and greatest maximum over every voxel a tied
        coordinate can round to;
      * clip floor (maximum within amb_clip * max(1, |clip|) of the clip, the
        reference's flag margin): 0, or a maximum inside that window;
      * grazing ray (chord within a hair of zero): a miss (-inf), 0, or the
        reference value.
    The last two (loose) kinds are also capped at max_loose_frac of the pixels."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fl = np.zeros(gpu.shape, dtype=np.int32) if flags is None else np.asarray(flags)
    tie = (fl & oracle.FLAG_NEAREST_AMBIG) > 0
    loose = (fl & (oracle.FLAG_MIPCLIP_AMBIG | oracle.FLAG_GRAZE_AMBIG)) > 0
    amb = tie | loose | ((fl & oracle.FLAGS_AMBIGUOUS) > 0)
    scale = np.maximum(1.0, np.abs(np.where(np.isfinite(ref), ref, 0.0)))
    strict = ~amb
    miss_g, miss_r = np.isneginf(gpu), np.isneginf(ref)
    assert np.array_equal(miss_g[strict], miss_r[strict]), "hit/miss pattern differs"
    hit = strict & ~miss_r
    diff = np.abs(gpu[hit] - ref[hit])
    rel = diff / scale[hit]
    worst = float(rel.max()) if rel.size else 0.0
    info = {"max_rel_err": worst, "max_abs_err": float(diff.max()) if diff.size else 0.0,
            "rms_abs_err": float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0,
            "n_ties": int(tie.sum()), "n_loose": int(loose.sum()), "n": int(gpu.size)}
    assert worst <= tol, info
    # nearest ties (and nothing looser): inside the interval of correct maxima
    only_tie = tie & ~loose
    if only_tie.any():
        assert bounds is not None, "nearest ties need the reference's bounds"
        b = np.asarray(bounds, dtype=np.float64)
        lo, hi = b[..., 0][only_tie], b[..., 1][only_tie]
        g = gpu[only_tie]
        sc = scale[only_tie]
        ok = (g >= np.maximum(lo, clip) - tol * sc) & (g <= hi + tol * sc) & (hi >= clip)
        ok |= (g == 0.0) & (lo < clip + tol * sc)  # floored: the maximum may lie below the clip
        assert ok.all(), (info, g[~ok][:5], lo[~ok][:5], hi[~ok][:5])
    if loose.any():
        g, r, sc = gpu[loose], ref[loose], scale[loose]
        near = np.isfinite(r) & (np.abs(g - r) <= tol * sc)
        ok = near | (g == 0.0) | (np.isneginf(g) & ((fl[loose] & oracle.FLAG_GRAZE_AMBIG) > 0))
        if math.isfinite(clip):
            # the reference floored its maximum to 0 or kept it; the unfloored
            # maximum lies within the flag's window around the clip
            win = amb_clip * max(1.0, abs(clip)) + tol * sc
            ok |= ((fl[loose] & oracle.FLAG_MIPCLIP_AMBIG) > 0) & (np.abs(g - clip) <= win)
        if bounds is not None:
            b = np.asarray(bounds, dtype=np.float64)
            lo, hi = b[..., 0][loose], b[..., 1][loose]
            ok |= np.isfinite(lo) & (g >= lo - tol * sc) & (g <= hi + tol * sc)
        assert ok.all(), (info, g[~ok][:5], r[~ok][:5])
        assert loose.mean() <= max_loose_frac, info
    return info


def wl_kwargs(wl, tf):
    """Reference keyword arguments for a workload (float32 TF rows promoted exactly)."""
    return dict(tf=np.asarray(tf, dtype=np.float64), v0=wl.v0, v1=wl.v1,
                clip=wl.clip_k * wl.cube.sigma, step=wl.step, ert=float(np.float32(wl.ert)))


def set_state(r, wl, tf, camera, clip=True):
    r.set_transfer_function(tf, wl.v0, wl.v1)
    r.set_noise_clip(wl.clip_k if clip else -math.inf, wl.cube.sigma)
    r.set_camera(camera)


def record(tag, info):
    """Print a comparison's errors and, when VR_PARITY_LOG names a file, append
    them to it as one JSON line (the per-image error table is built from it)."""
    print(tag, info, flush=True)
    path = os.environ.get("VR_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": tag, **{k: v for k, v in info.items()}}) + "\n")
