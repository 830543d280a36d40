#!/usr/bin/env python3
"""Renderer benchmark: Gsamples/s and ms/frame for 1024x1024 perspective views of
the 512x512x1024 float32 noisy spectral cube (noise sigma 1 plus 200 Gaussian
sources), trilinear sampling, step 0.5 voxel, ramp transfer function clipped
below 3 sigma, emission-absorption compositing with early termination at 0.99,
32^3 bricks with 8^3-cell empty-space skipping.

One step = one frame: the whole hot path (ray set-up, brick traversal, skip
tests, sampling, classification, compositing, store) for one orbit view; the
16 seeded views are cycled.  Inputs are resident in HBM before timing starts.
Prints ONE JSON line.  Only one GPU is supported.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# Vector-ALU issue of the whole chip without packed FP32 (which this build
# disables): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second.
PEAK_VALU_LANE_INSTR = 256 * 4 * 16 * 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_render_full512_traffic.txt")
L2_FILE = os.path.join(ROOT, "profiles", "k_render_full512_l2.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "k_render_full512_sq.txt")
# sources that define the render kernels: committed counter summaries carry
# their digest and are used only while it matches
KERNEL_SOURCES = ["vr_common.h", "vr_dev.h", "vr_render.h",
                  "vr_render_ea_f32.hip", "vr_render_ea_f16.hip", "vr_render_ea_bf16.hip",
                  "vr_render_mip_f32.hip", "vr_render_mip_f16.hip", "vr_render_mip_bf16.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads():
    """Host threads for CPU work: every core this process may run on."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(vol, tf, wl, cams, W, H, mode, budget_s=12.0, max_frames=64):
    """The FP64 reference timed on the host cores over whole frames (the
    workload's views in turn) until ~budget_s."""
    import numpy as np

    import oracle
    th = cpu_threads()
    total, t_all, nviews = 0, 0.0, 0
    for i in range(max_frames):
        cam = cams[i % len(cams)]
        t0 = time.perf_counter()
        res = oracle.render(vol, mode=oracle.EA if mode == "ea" else oracle.MIP,
                            tf=tf.astype(np.float64), v0=wl.v0, v1=wl.v1, clip=wl.clip_k,
                            step=wl.step, ert=float(np.float32(wl.ert)), camera=cam, width=W,
                            height=H, threads=th)
        t_all += time.perf_counter() - t0
        total += int(res["n_nominal"].sum())
        nviews += 1
        if t_all >= budget_s:
            break
    return {"value": total / t_all / 1e9, "unit": "Gsamples/s", "cores": th, "kind": "oracle",
            "sample": "%d full %dx%d frame(s) of the same workload (its %d views in turn), %.1f s"
                      % (nviews, W, H, len(cams), t_all),
            "host_nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "ms_per_frame": round(t_all / nviews * 1e3, 1)}


def serving_leg(n_requests=2000, n_warm=200, loads=(0.5, 0.7, 0.9), seed=4242):
    """Serving form: 8 FP16 cubes (sizes drawn per axis from 128..1024 x
    128..1024 x 128..512, noise plus density-matched sources) registered from
    pinned host memory, view requests with random orbit cameras, image sizes
    {256, 512, 1024, 2048}^2 and EA/MIP 50/50, served with continuous batching.
    Two memory budgets: (i) unconstrained (every cube resident after its first
    use) and (ii) half of the cubes' total device bytes, so that cubes are
    admitted and evicted while requests run.  For each budget a closed loop
    (all requests at once) gives the saturation throughput; then, after
    n_warm warm-up requests, n_requests arrive as a Poisson process at each
    load x that rate and the server-side latency (arrival to completion) is
    reported as p50/p99."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1001_2049_amd import Renderer

    specs = synth.serving_cubes(8)
    codes, t_gen = [], 0.0
    for sp in specs:
        t0 = time.perf_counter()
        vol = synth.cube(sp, threads=cpu_threads())
        t_gen += time.perf_counter() - t0
        c = torch.from_numpy(oracle.to_f16_bits(vol).view(np.float16)).pin_memory()
        codes.append(c)
        del vol
    log("serving: 8 cubes generated in %.1f s" % t_gen)
    tf = synth.ramp_tf(256, 1.0)
    rng = np.random.default_rng(seed)
    sizes = [256, 512, 1024, 2048]
    total_req = n_warm + n_requests
    plan = []
    for i in range(total_req):
        ci = int(rng.integers(0, 8))
        sz = sizes[int(rng.integers(0, 4))]
        mode = "ea" if rng.random() < 0.5 else "mip"
        sp = specs[ci]
        cam = synth.orbit_camera(sp.nx, sp.ny, sp.nz, float(rng.uniform(0, 2 * math.pi)),
                                 float(rng.uniform(-math.pi / 4, math.pi / 4)))
        plan.append((ci, sz, mode, cam))
    gaps_unit = rng.exponential(1.0, size=total_req)
    # outputs: a ring per (size, mode) class, longer than the requests in flight
    max_batch, max_inflight = 64, 2
    ring = max_batch * max_inflight + 16

    def make_outputs(r):
        pools, count, outs = {}, {}, []
        for ci, sz, mode, cam in plan:
            k = (sz, mode)
            lst = pools.setdefault(k, [])
            idx = count.get(k, 0)
            count[k] = idx + 1
            if len(lst) < ring:
                lst.append(r.output(sz, sz, mode))
            outs.append(lst[idx % ring])
        return outs

    res = {"requests": n_requests, "warmup_requests": n_warm, "loads": list(loads),
           "cubes": [[sp.nx, sp.ny, sp.nz] for sp in specs], "storage": "f16", "budgets": {}}
    samples = None
    total_bytes = None
    for budget_name in ("unconstrained", "half"):
        budget = 0 if budget_name == "unconstrained" else total_bytes // 2
        r = Renderer(0, budget_bytes=budget)
        try:
            cubes = [r.register(c, "f16", src_dtype="f16") for c in codes]
            if total_bytes is None:
                total_bytes = 0
                for c in cubes:
                    inf = r.info(c)
                    slots = inf.bricks_x * inf.bricks_y * inf.bricks_z
                    total_bytes += (inf.pool_bytes + 255) // 256 * 256 + (slots * 512 + 255) // 256 * 256
            r.set_transfer_function(tf, 3.0, 50.0)
            r.set_noise_clip(3.0, 1.0)
            outs = make_outputs(r)
            reqs = [r.request(cubes[ci], cam, sz, sz, out, mode=mode, clip=3.0)
                    for (ci, sz, mode, cam), out in zip(plan, outs)]
            if samples is None:
                # nominal samples per request (untimed pass with counters)
                samples = []
                for k in range(0, total_req, 32):
                    samples += [st["samples_nominal"] for st in r.render_batch(reqs[k:k + 32], stats=True)]
                torch.cuda.synchronize()
                # the plain renderer, one request after another (first 256 requests)
                t0 = time.perf_counter()
                for (ci, sz, mode, cam), out in list(zip(plan, outs))[:256]:
                    r.set_camera(cam)
                    r.render(cubes[ci], sz, sz, mode=mode, out=out)
                torch.cuda.synchronize()
                res["plain_sequential_gsamples_per_s"] = round(
                    float(sum(samples[:256])) / (time.perf_counter() - t0) / 1e9, 3)
            r.server_start(max_batch_requests=max_batch, max_batch_tiles=4096,
                           max_inflight=max_inflight, use_graphs=1)
            cell = {"budget_bytes": int(budget), "total_cube_bytes": int(total_bytes)}
            try:
                for t in [r.submit(q) for q in reqs[:n_warm]]:
                    r.wait(t, timeout_s=300)
                timed = reqs[n_warm:]
                tot = float(sum(samples[n_warm:]))
                t0 = time.perf_counter()
                tickets = [r.submit(q) for q in timed]
                for t in tickets:
                    r.wait(t, timeout_s=600)
                t_sat = time.perf_counter() - t0
                rate_sat = len(timed) / t_sat
                cell["saturation_requests_per_s"] = round(rate_sat, 2)
                cell["saturation_gsamples_per_s"] = round(tot / t_sat / 1e9, 3)
                log("serving %s: saturation %.1f requests/s" % (budget_name, rate_sat))
                for load in loads:
                    lam = load * rate_sat
                    lat = []
                    for phase, part in (("warm", reqs[:n_warm]), ("timed", timed)):
                        g = gaps_unit[:len(part)] / lam
                        t0 = time.perf_counter()
                        t_next = t0
                        tickets = []
                        for q, gap in zip(part, g):
                            t_next += gap
                            d = t_next - time.perf_counter()
                            if d > 0:
                                time.sleep(d)
                            tickets.append(r.submit(q))
                        l = [r.wait(t, timeout_s=600) for t in tickets]
                        if phase == "timed":
                            lat = l
                            t_open = time.perf_counter() - t0
                    lat_ms = np.asarray(lat) * 1e3
                    cell["load_%.1f" % load] = {
                        "rate_per_s": round(lam, 2),
                        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
                        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
                        "latency_ms_max": round(float(lat_ms.max()), 3),
                        "gsamples_per_s": round(tot / t_open / 1e9, 3)}
                    log("serving %s load %.1f: p50 %.2f ms p99 %.2f ms" % (
                        budget_name, load, cell["load_%.1f" % load]["latency_ms_p50"],
                        cell["load_%.1f" % load]["latency_ms_p99"]))
            finally:
                r.server_stop()
            cell["memory"] = r.memory_stats()
            res["budgets"][budget_name] = cell
        finally:
            r.close()
            torch.cuda.empty_cache()
    res["samples_total"] = float(sum(samples[n_warm:]))
    return res


def copy_bandwidth_gbs(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate of nbytes (read plus write bytes per second),
    the stream bandwidth this HBM actually reaches, as a second reference
    beside the 8 TB/s specification."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def kernel_source_digest():
    """SHA-256 over the render kernels' sources, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1001_2049_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def read_summary(path):
    kv = {}
    try:
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
    except OSError:
        return None
    return kv if kv.get("kernel_source_sha256") == kernel_source_digest() else None


def measured_valu(kernel_name, width, samples, kernel_ms):
    """Vector-ALU roofline of the render kernel from the committed SQ counter
    summary: wave-level VALU instructions x 64 lanes per nominal sample, over
    this run's kernel time, against the chip's non-packed issue rate."""
    kv = read_summary(SQ_FILE)
    if kv is None or kv.get("kernel") != kernel_name or int(kv.get("image_width", "0")) != width:
        return None
    per = float(kv["valu_lane_instr_per_sample"])
    achieved = per * samples / (kernel_ms * 1e-3)
    return {"bound": "alu", "lane_instr_per_sample": per,
            "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_VALU_LANE_INSTR / 1e12, 2),
            "unit": "T lane-instr/s", "frac": round(achieved / PEAK_VALU_LANE_INSTR, 4),
            "lds_instr_per_sample": float(kv.get("lds_instr_per_sample", "nan")),
            "lds_bank_conflict_cycles_per_lds_instr": float(kv.get("lds_bank_conflict_cycles_per_lds_instr", "nan"))}


def measured_traffic(kernel_name, width):
    """HBM bytes per launch of the render kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size), or None when that summary was taken on other kernel source."""
    kv = read_summary(TRAFFIC_FILE)
    if kv is None:
        return None
    if kv.get("kernel") != kernel_name or int(kv.get("image_width", "0")) != width:
        return None
    return float(kv["hbm_bytes_per_launch"])


def measured_l2(kernel_name, width, kernel_ms):
    """L2 read traffic of the render kernel from the committed rocprofv3 TCC
    counter summary, as bytes per launch over this run's measured kernel time,
    or None when that summary was taken on other kernel source."""
    kv = read_summary(L2_FILE)
    if kv is None or kv.get("kernel") != kernel_name:
        return None
    if width != 1024:
        return None
    read_bytes = float(kv["l2_read_bytes_per_launch"])
    return {"read_bytes_per_launch": read_bytes, "hit_rate": float(kv["l2_hit_rate"]),
            "achieved": round(read_bytes / (kernel_ms * 1e-3) / 1e9, 1), "unit": "GB/s"}


def time_frames(r, cube, cams, W, H, mode, interp, step, ert, reps=1):
    """Mean kernel ms per frame and nominal samples per frame over the views
    (events on the launch stream around each render, after one warm-up view)."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    out = r.output(W, H, mode)
    kw = dict(mode=mode, interp=interp, step=step, ert=ert, out=out)
    nominal = []
    for cam in cams:
        r.set_camera(cam)
        _, st = r.render(cube, W, H, stats=True, **kw)
        nominal.append(st["samples_nominal"])
    r.set_camera(cams[0])
    r.render(cube, W, H, **kw)
    ms = []
    for _ in range(reps):
        for cam in cams:
            r.set_camera(cam)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            r.render(cube, W, H, **kw)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
    m = float(np.mean(ms))
    return {"ms_per_frame": round(m, 4), "gsamples_per_s": round(float(np.mean(nominal)) / m / 1e6, 2),
            "samples_per_frame": float(np.mean(nominal))}


def variants(r, cube_f32, vol, wl, tf, cams, args):
    """The other configurations of the full-size workload, each timed over the
    16 orbit views: FP16 / BF16 storage (EA at 1024^2 and 2048^2), and MIP
    (trilinear and nearest) on the FP32 cube at 1024^2; reported beside the
    FP32 EA headline on the same GPU."""
    out = {}
    kw = dict(step=wl.step, ert=wl.ert)
    out["f32_mip_trilinear_1024"] = time_frames(r, cube_f32, cams, 1024, 1024, "mip", "trilinear", **kw)
    out["f32_mip_nearest_1024"] = time_frames(r, cube_f32, cams, 1024, 1024, "mip", "nearest", **kw)
    out["f32_ea_2048"] = time_frames(r, cube_f32, cams, 2048, 2048, "ea", "trilinear", **kw)
    for storage in ("f16", "bf16"):
        c = r.upload(vol, storage)
        try:
            for size in (1024, 2048):
                out["%s_ea_%d" % (storage, size)] = time_frames(r, c, cams, size, size, "ea",
                                                                 "trilinear", **kw)
            out["%s_mip_trilinear_1024" % storage] = time_frames(r, c, cams, 1024, 1024, "mip",
                                                                  "trilinear", **kw)
        finally:
            r.release(c)
    return out


def features(r, cube_f32, vol, wl, cams):
    """The rows beyond the plain renderer, timed on the full-size FP32 cube at
    1024^2 (view 0, HIP events on the launch stream):
    sub-cubes: the cube split into 8 windows of 128 planes along z
    (512x512x128 each), one partial per window and their integration,
    against the whole render, ERT off so both images agree to rounding;
    noise: per-channel median / MAD over the 1024 channels of 512^2 (cube in
    device memory) and the scaled upload;
    streamed: the cube registered under half its bricks' bytes, frame time;
    progressive: the first call (which builds the cube's coarse levels), then
    the coarse-to-fine levels 4 .. 0 of another view."""
    import numpy as np
    import torch

    import synth
    W = H = 1024
    res = {}
    stream = torch.cuda.current_stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        v = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), v

    r.set_camera(cams[0])
    kw = dict(mode="ea", step=wl.step, ert=2.0)
    whole = r.output(W, H, "ea")
    r.render(cube_f32, W, H, out=whole, **kw)
    whole_ms, _ = timed(lambda: r.render(cube_f32, W, H, out=whole, **kw))
    nz = wl.cube.nz
    edges = list(range(0, nz + 1, nz // 8))
    parts = [r.output(W, H, "ea") for _ in range(8)]
    comp = r.output(W, H, "ea")

    def split():
        for k in range(8):
            r.render_subcube(cube_f32, W, H, 2, edges[k], edges[k + 1], out=parts[k], **kw)
        return None
    split()
    split_ms, _ = timed(split)
    comp_ms, _ = timed(lambda: r.composite(parts, 2, W, H, mode="ea", out=comp))
    diff = float((comp - whole).abs().max().item())
    res["subcube_split8_z"] = {"whole_ms": round(whole_ms, 3), "partials_ms": round(split_ms, 3),
                               "composite_ms": round(comp_ms, 3),
                               "max_abs_diff_vs_whole": diff}

    dev = torch.from_numpy(vol).cuda()
    r.estimate_channel_noise(dev)
    noise_ms, (med, mad, sig) = timed(lambda: r.estimate_channel_noise(dev))
    up_ms, c2 = timed(lambda: r.upload_scaled(dev, np.maximum(sig, 1e-6), "f32"))
    r.release(c2)
    del dev
    torch.cuda.empty_cache()
    res["noise"] = {"channels": int(nz), "estimate_ms": round(noise_ms, 3),
                    "scaled_upload_ms": round(up_ms, 3),
                    "sigma_mean": round(float(np.mean(sig)), 4)}

    # the same cube registered from host memory under a budget of half its
    # bricks: streamed, each frame uploads the bricks over PCIe as sub-cubes of
    # brick layers (wall-clock, median of 3; the first frame also bricks the
    # cube into pinned host memory)
    from paper_1001_2049_amd import Renderer
    budget = int(r.info(cube_f32).pool_bytes // 2)
    rs = Renderer(0, budget_bytes=budget)
    try:
        rs.set_transfer_function(synth.ramp_tf(256, wl.kappa_max), wl.v0, wl.v1)
        rs.set_noise_clip(wl.clip_k, wl.cube.sigma)
        rs.set_camera(cams[0])
        sc = rs.register(vol, "f32")
        simg = rs.output(W, H, "ea")

        def wall(fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0)
        first = wall(lambda: rs.render(sc, W, H, out=simg, **kw))
        frames = sorted(wall(lambda: rs.render(sc, W, H, out=simg, **kw)) for _ in range(3))
        res["streamed"] = {"budget_bytes": budget, "pool_bytes": int(rs.info(sc).pool_bytes),
                           "first_frame_ms": round(first, 1), "frame_ms": round(frames[1], 2),
                           "resident_ms": round(whole_ms, 3),
                           "max_abs_diff_vs_resident": float((simg - whole).abs().max().item())}
        # its progressive loop: the first call builds resident coarse levels
        # from the pinned bricks, then levels 2, 1 and the streamed level 0
        pout = rs.output(W, H, "ea")
        pk = dict(max_level=3, mode="ea", step=wl.step, ert=wl.ert)
        got = []
        t_first = wall(lambda: got.append(rs.render_progressive(sc, W, H, pout, 0.01, **pk)))
        lv = [{"level": got[0]["level"], "ms": round(got[0]["ms"], 3), "level_cube": got[0]["level_cube"],
               "call_ms_with_level_build": round(t_first, 1)}]
        for _ in range(4):
            inf = rs.render_progressive(sc, W, H, pout, 0.01, **pk)
            if inf["converged"]:
                break
            lv.append({"level": inf["level"], "ms": round(inf["ms"], 3), "level_cube": inf["level_cube"]})
        res["streamed"]["progressive"] = lv
    finally:
        rs.close()
    torch.cuda.empty_cache()

    # the first call on a cube builds its coarse levels (2x2x2 block means)
    out = r.output(W, H, "ea")
    pk = dict(max_level=4, mode="ea", step=wl.step, ert=wl.ert)
    first_ms, info = timed(lambda: r.render_progressive(cube_f32, W, H, out, 0.01, **pk))
    r.set_camera(cams[1])
    levels = []
    for _ in range(6):
        info = r.render_progressive(cube_f32, W, H, out, 0.01, **pk)
        if info["converged"]:
            break
        levels.append({"level": info["level"], "ms": round(info["ms"], 3),
                       "samples": int(info["samples_nominal"]), "level_cube": info["level_cube"]})
    res["progressive"] = {"first_call_with_level_build_ms": round(first_ms, 3), "levels": levels}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--mode", default="ea", choices=["ea", "mip"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--size", type=int, default=1024, help="image width = height")
    ap.add_argument("--no-skip", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-features", action="store_true",
                    help="skip the sub-cube, noise and progressive timings (also off with --no-variants)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus %d requested); the renderer has no "
              "multi-GPU path" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1001_2049_amd import Renderer

    wl = synth.full()
    W = H = args.size
    log("generating %dx%dx%d cube" % (wl.cube.nx, wl.cube.ny, wl.cube.nz))
    vol = synth.cube(wl.cube, threads=cpu_threads())
    tf = synth.ramp_tf(256, wl.kappa_max)
    cams = [synth.orbit_camera(wl.cube.nx, wl.cube.ny, wl.cube.nz, th, ph)
            for th, ph in synth.orbit_angles(wl.extra["camera_seed"], wl.extra["n_views"])]

    r = Renderer(0)
    t0 = time.perf_counter()
    cube = r.upload(vol, args.storage)
    log("upload %.3f s" % (time.perf_counter() - t0))
    r.set_transfer_function(tf, wl.v0, wl.v1)
    r.set_noise_clip(wl.clip_k, wl.cube.sigma)
    out = r.output(W, H, args.mode)
    kw = dict(mode=args.mode, step=wl.step, ert=wl.ert, use_skip=not args.no_skip, out=out)

    # per-view sample counts (untimed pass with counters)
    nominal, executed = [], []
    for cam in cams:
        r.set_camera(cam)
        _, st = r.render(cube, W, H, stats=True, **kw)
        nominal.append(st["samples_nominal"])
        executed.append(st["samples_exec"])
    log("nominal samples/frame: mean %.4g" % np.mean(nominal))

    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        r.set_camera(cams[k % len(cams)])
        r.render(cube, W, H, **kw)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        r.set_camera(cams[k % len(cams)])
        evs[k][0].record(stream)
        r.render(cube, W, H, **kw)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in evs]
    samples = sum(nominal[k % len(cams)] for k in range(args.steps))
    samples_exec = sum(executed[k % len(cams)] for k in range(args.steps))
    gsps = samples / wall / 1e9
    avg_ms = float(np.mean(kernel_ms))

    elem = {"f32": 4, "f16": 2, "bf16": 2}[args.storage]
    cube_bytes = wl.cube.nx * wl.cube.ny * wl.cube.nz * elem
    img_bytes = W * H * (16 if args.mode == "ea" else 4)
    alg_bytes = cube_bytes + img_bytes
    frame_s = avg_ms * 1e-3
    hbm_achieved = alg_bytes / frame_s / 1e9
    kernel_name = "k_render<%s,%s,trilinear>" % (args.mode, args.storage)
    traffic = measured_traffic(kernel_name, W)
    copy_gbs = copy_bandwidth_gbs()

    res = {
        "metric": "Gsamples/s (nominal samples per second), 1024x1024 view of 512x512x1024 cube",
        "value": round(gsps, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic (seeded noise + 200 Gaussian sources)",
        "config": {
            "workload": "full-512x512x1024 %s cube, %dx%d perspective orbit views (16 seeded), "
                        "%s trilinear, step 0.5, ERT 0.99, ramp TF [3,50] clipped at 3 sigma, "
                        "32^3 bricks, 8^3 skip cells%s" % (args.storage, W, H, args.mode.upper(),
                                                          "" if not args.no_skip else ", skip off"),
            "image": [W, H],
            "cube": [wl.cube.nx, wl.cube.ny, wl.cube.nz],
            "mode": args.mode,
            "samples_per_frame": float(np.mean(nominal)),
            "executed_samples_per_frame": float(samples_exec / args.steps),
            "executed_gsamples_per_s": round(samples_exec / wall / 1e9, 3),
            "kernel_ms_mean": round(avg_ms, 4),
            "kernel_ms_median": round(float(np.median(kernel_ms)), 4),
            "kernel_ms_p90": round(float(np.percentile(kernel_ms, 90)), 4),
        },
        # The HBM roofline: the compulsory bytes of one frame (the cube read once
        # plus the image written) over the frame's kernel time, against 8 TB/s.
        # traffic: HBM bytes per launch from the committed rocprofv3 counters.
        "roofline": {
            "bound": "hbm",
            "achieved": round(hbm_achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(hbm_achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": kernel_name,
            "algorithmic_bytes_per_launch": alg_bytes,
            # the same against the device-to-device copy rate measured in this run
            "copy_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(hbm_achieved / copy_gbs, 4),
        },
        # vector-ALU issue (wave instructions x 64 lanes, from committed SQ counters)
        "valu_roofline": measured_valu(kernel_name, W, samples / args.steps, avg_ms),
        # L2 reads per launch (TCC counters) over this run's kernel time
        "l2": measured_l2(kernel_name, W, avg_ms),
    }
    if not args.no_variants and args.storage == "f32" and W == 1024 and args.mode == "ea":
        log("configuration variants")
        res["variants"] = variants(r, cube, vol, wl, tf, cams, args)
    if (not args.no_features and not args.no_variants and args.storage == "f32" and W == 1024
            and args.mode == "ea"):
        log("sub-cubes, noise estimation, progressive levels")
        res["features"] = features(r, cube, vol, wl, cams)
    if not args.no_cpu_baseline:
        log("timing the CPU reference")
        res["cpu_baseline"] = cpu_baseline(vol, tf, wl, cams, W, H, args.mode)
    r.close()
    del r
    if not args.no_serving:
        log("serving leg")
        res["serving"] = serving_leg(args.serving_requests, args.serving_warmup)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
