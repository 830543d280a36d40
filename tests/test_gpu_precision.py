"""Precision form on the GPU: cubes stored as FP16 / BF16 codes of v/sigma,
decoded and interpolated, classified and composited in FP32.

* gate: GPU image on 16-bit storage vs the FP64 reference on the ORIGINAL
  float32 cube (the error includes the storage rounding) -> 4e-3 per channel;
  max and RMS error are printed per image;
* arithmetic: GPU vs the reference on the DECODED codes -> the FP32 tolerance,
  which isolates kernel errors from storage rounding;
* layout: the brick pool's bytes equal the host's round-to-nearest-even codes
  at every stored voxel (edge-clamped apron included) and the cell min/max
  tables equal a brute-force min/max over each cell's 9^3 halo;
* scaling: data and sigma both multiplied by 2^m give bit-identical images
  (EA) and exactly 2^m times the MIP image.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_16, TOL_F32, compare_ea, compare_mip, record, ref_render, wl_kwargs

pytestmark = pytest.mark.gpu

CODES = {"f16": oracle.F16, "bf16": oracle.BF16}


def codes_of(vol, storage, sigma=1.0):
    x = (np.asarray(vol, dtype=np.float32) / np.float32(sigma)).astype(np.float32)
    return oracle.to_f16_bits(x) if storage == "f16" else oracle.to_bf16_bits(x)


def hip_to_host(ptr, nbytes):
    """Copy device memory the library owns into a host buffer (hipMemcpy D2H)."""
    import torch
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(nbytes, dtype=np.uint8)
    rc = hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), nbytes, 2)
    assert rc == 0, rc
    return out


@pytest.fixture(scope="module")
def rend():
    import torch
    from paper_1001_2049_amd import Renderer
    r = Renderer(0)
    yield r
    r.close()
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def tiny_cube():
    wl = synth.tiny()
    return wl, synth.cube(wl.cube), synth.ramp_tf(256, wl.kappa_max)


def report(tag, info):
    record(tag, info)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("mode", ["ea", "mip"])
@pytest.mark.parametrize("view", ["z", "orbit"])
def test_tiny_gate_and_arithmetic(rend, tiny_cube, storage, mode, view):
    import torch
    wl, vol, tf = tiny_cube
    cube = rend.upload(vol, storage)
    try:
        if view == "z":
            cam = synth.axis_camera(64, 64, 128, "z", 256, 256)
        else:
            cam = synth.orbit_camera(64, 64, 128, 0.9, 0.35)
        W = H = 256
        rend.set_transfer_function(tf, wl.v0, wl.v1)
        rend.set_noise_clip(wl.clip_k, 1.0)
        rend.set_camera(cam)
        img = rend.render(cube, W, H, mode=mode)
        torch.cuda.synchronize()
        got = img.cpu().numpy().astype(np.float64)
        kw = wl_kwargs(wl, tf)
        # gate: against the original float32 values; the ERT and clip ambiguity
        # margins are widened to the storage rounding (a decision that storage
        # rounding can flip has several correct results)
        ref = ref_render(vol, kw, cam, W, H, mode, "trilinear", amb_ert=TOL_16, amb_clip=TOL_16)
        if mode == "ea":
            info = compare_ea(got, ref["image"], TOL_16, ref["flags"], max_ambiguous_frac=0.05)
        else:
            info = compare_mip(got, ref["image"], TOL_16, ref["flags"], ref.get("bounds"),
                               clip=wl.clip_k, amb_clip=TOL_16)
        report("gate %s %s %s" % (storage, mode, view), info)
        # arithmetic: against the decoded codes
        dec = ref_render(codes_of(vol, storage), kw, cam, W, H, mode, "trilinear",
                         vox_dtype=CODES[storage])
        if mode == "ea":
            info = compare_ea(got, dec["image"], TOL_F32, dec["flags"])
        else:
            info = compare_mip(got, dec["image"], TOL_F32, dec["flags"], dec.get("bounds"),
                               clip=wl.clip_k)
        report("arith %s %s %s" % (storage, mode, view), info)
    finally:
        rend.release(cube)


@pytest.mark.parametrize("storage", ["f16", "bf16", "f32"])
def test_pool_layout_and_cell_tables(rend, storage):
    """Every stored element of every slot (the 33^3 brick, its apron and the
    padding) equals the host's storage code of the edge-clamped voxel, at the
    position the documented line layout gives; the cell tables equal a
    brute-force min/max over each cell's 9^3 halo."""
    nx, ny, nz = 45, 70, 33
    rng = np.random.default_rng(7)
    vol = (rng.standard_normal((nz, ny, nx)) * 3.0).astype(np.float32)
    sigma = 0.5 if storage != "f32" else 1.0
    cube = rend.upload(vol, storage, sigma_scale=sigma)
    try:
        inf = rend.info(cube)
        B = inf.brick
        assert (inf.bricks_x, inf.bricks_y, inf.bricks_z) == (2, 3, 2)
        esz = 4 if storage == "f32" else 2
        cv = 16 // esz
        xch = inf.x_chunks
        assert xch * cv >= B + 1
        nslots = inf.bricks_x * inf.bricks_y * inf.bricks_z
        slot_elems = 17 * 9 * xch * 8 * cv
        assert inf.brick_stride >= slot_elems * esz and inf.brick_stride % 256 == 0
        raw = hip_to_host(inf.pool, nslots * inf.brick_stride)
        if storage == "f32":
            want_all = (vol / np.float32(sigma)).astype(np.float32)
            dt = np.float32
        else:
            want_all = codes_of(vol, storage, sigma)
            dt = np.uint16
        mm = hip_to_host(inf.cell_minmax, nslots * 64 * 2 * 4).view(np.float32).reshape(nslots, 64, 2)
        if storage == "f32":
            dec_all = want_all.astype(np.float64)
        else:
            dec_all = oracle.decode_bits(want_all, CODES[storage])
        # element offset of local (lx, ly, lz): the documented formula
        lx = np.arange(xch * cv)
        ly = np.arange(36)
        lz = np.arange(34)
        ox = (lx // cv) * 8 * cv + lx % cv
        oy = (ly // 4) * xch * 8 * cv + (ly % 4) * cv
        oz = (lz // 2) * 9 * xch * 8 * cv + (lz % 2) * 4 * cv
        off = oz[:, None, None] + oy[None, :, None] + ox[None, None, :]
        assert np.array_equal(np.sort(off.ravel()), np.arange(slot_elems))  # a bijection
        for bz in range(inf.bricks_z):
            for by in range(inf.bricks_y):
                for bx in range(inf.bricks_x):
                    slot = (bz * inf.bricks_y + by) * inf.bricks_x + bx
                    base = slot * inf.brick_stride
                    sv = raw[base: base + slot_elems * esz].view(dt)[off]
                    gz = np.minimum(lz + B * bz, nz - 1)
                    gy = np.minimum(ly + B * by, ny - 1)
                    gx = np.minimum(lx + B * bx, nx - 1)
                    want = want_all[np.ix_(gz, gy, gx)]
                    assert np.array_equal(np.ascontiguousarray(sv).view(np.uint8),
                                          np.ascontiguousarray(want).view(np.uint8)), slot
                    dec = dec_all[np.ix_(gz[:33], gy[:33], gx[:33])]
                    for c in range(64):
                        cx, cy, cz = c % 4, (c // 4) % 4, c // 16
                        blk = dec[8 * cz: 8 * cz + 9, 8 * cy: 8 * cy + 9, 8 * cx: 8 * cx + 9]
                        assert mm[slot, c, 0] == np.float32(blk.min()), (slot, c)
                        assert mm[slot, c, 1] == np.float32(blk.max()), (slot, c)
    finally:
        rend.release(cube)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_power_of_two_scaling_bit_identical(rend, tiny_cube, storage):
    import torch
    wl, vol, tf = tiny_cube
    cam = synth.orbit_camera(64, 64, 128, 2.1, -0.3)
    rend.set_camera(cam)
    outs = {}
    for m in (0, 3):
        f = float(2 ** m)
        cube = rend.upload((vol * np.float32(f)).astype(np.float32), storage, sigma_scale=f)
        try:
            rend.set_transfer_function(tf, wl.v0 * f, wl.v1 * f)
            rend.set_noise_clip(wl.clip_k, f)
            ea = rend.render(cube, 160, 120, mode="ea")
            mip = rend.render(cube, 160, 120, mode="mip")
            torch.cuda.synchronize()
            outs[m] = (ea.cpu().numpy(), mip.cpu().numpy())
        finally:
            rend.release(cube)
    assert np.array_equal(outs[0][0].view(np.uint32), outs[3][0].view(np.uint32))
    assert np.array_equal((outs[0][1] * np.float32(8.0)).view(np.uint32), outs[3][1].view(np.uint32))


@pytest.mark.parametrize("storage,size", [("f16", 1024), ("bf16", 1024), ("f16", 2048),
                                          ("bf16", 2048)])
def test_full_cube_sampled_gate(rend, full_workload, storage, size):
    """The full-size cube stored in 16 bits, 1024^2 / 2048^2 perspective views:
    sampled pixels vs the reference on the original float32 values (gate) and
    on the decoded codes (arithmetic)."""
    import torch
    wl, vol, tf = full_workload
    cube = rend.upload(vol, storage)
    try:
        cams = [synth.orbit_camera(512, 512, 1024, th, ph)
                for th, ph in synth.orbit_angles(wl.extra["camera_seed"], 2)]
        kw = wl_kwargs(wl, tf)
        codes = codes_of(vol, storage)
        rend.set_transfer_function(tf, wl.v0, wl.v1)
        rend.set_noise_clip(wl.clip_k, 1.0)
        for vi, cam in enumerate(cams):
            rend.set_camera(cam)
            for mode in ("ea", "mip"):
                img = rend.render(cube, size, size, mode=mode)
                torch.cuda.synchronize()
                got_img = img.cpu().numpy()
                px = synth.pixel_subset(100 + vi, size, size, 1500)
                got = got_img[px[:, 1], px[:, 0]].astype(np.float64)
                ref = ref_render(vol, kw, cam, size, size, mode, "trilinear", pixels=px,
                                 amb_ert=TOL_16, amb_clip=TOL_16)
                dec = ref_render(codes, kw, cam, size, size, mode, "trilinear", pixels=px,
                                 vox_dtype=CODES[storage])
                if mode == "ea":
                    g = compare_ea(got, ref["values"], TOL_16, ref["flags"], max_ambiguous_frac=0.05)
                    a = compare_ea(got, dec["values"], TOL_F32, dec["flags"])
                else:
                    g = compare_mip(got, ref["values"], TOL_16, ref["flags"], ref.get("bounds"),
                                    clip=wl.clip_k, amb_clip=TOL_16)
                    a = compare_mip(got, dec["values"], TOL_F32, dec["flags"], dec.get("bounds"),
                                    clip=wl.clip_k)
                report("full gate %s %d view%d %s" % (storage, size, vi, mode), g)
                report("full arith %s %d view%d %s" % (storage, size, vi, mode), a)
    finally:
        rend.release(cube)


def test_full_cube_2048_whole_frame(rend, full_workload):
    """One whole 2048^2 EA frame of the full-size cube stored as FP16 against
    the reference on every pixel: on the decoded codes (the renderer's own
    arithmetic, float32 tolerance) and on the original float32 values (the
    storage gate).  The reference's time for the whole frame is reported."""
    import os
    import time

    import torch
    wl, vol, tf = full_workload
    size = 2048
    cube = rend.upload(vol, "f16")
    try:
        cam = synth.orbit_camera(512, 512, 1024, *synth.orbit_angles(wl.extra["camera_seed"], 1)[0])
        kw = wl_kwargs(wl, tf)
        rend.set_transfer_function(tf, wl.v0, wl.v1)
        rend.set_noise_clip(wl.clip_k, 1.0)
        rend.set_camera(cam)
        img = rend.render(cube, size, size, mode="ea")
        torch.cuda.synchronize()
        got = img.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        dec = ref_render(codes_of(vol, "f16"), kw, cam, size, size, "ea", "trilinear",
                         vox_dtype=CODES["f16"], threads=os.cpu_count())
        t_ref = time.perf_counter() - t0
        ref = ref_render(vol, kw, cam, size, size, "ea", "trilinear", amb_ert=TOL_16, amb_clip=TOL_16,
                         threads=os.cpu_count())
        a = compare_ea(got, dec["image"], TOL_F32, dec["flags"])
        g = compare_ea(got, ref["image"], TOL_16, ref["flags"], max_ambiguous_frac=0.05)
        a["oracle_s"] = t_ref
        a["oracle_threads"] = os.cpu_count()
        a["nominal_samples"] = int(dec["n_nominal"].sum())
        report("whole frame arith f16 2048 view0 ea", a)
        report("whole frame gate f16 2048 view0 ea", g)
    finally:
        rend.release(cube)
