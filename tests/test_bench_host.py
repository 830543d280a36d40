"""Host-side checks of bench.py (no GPU): the committed counter summaries in
profiles/ belong to the render kernels' current sources (otherwise the bench
would report no traffic), their derived figures agree with their raw
counters, and a request for several GPUs is refused before anything touches
a device."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_summaries_match_current_kernel_sources():
    for path in (bench.TRAFFIC_FILE, bench.L2_FILE, bench.SQ_FILE):
        kv = bench.read_summary(path)
        assert kv is not None, "%s was taken on other kernel sources" % os.path.basename(path)
        assert kv["kernel"] == "k_render<ea,f32,trilinear>"


def test_traffic_summary_is_consistent():
    kv = bench.read_summary(bench.TRAFFIC_FILE)
    fetch, write = float(kv["fetch_kib_per_launch"]), float(kv["write_kib_per_launch"])
    fs, ws = float(kv["fetch_scale"]), float(kv["write_scale"])
    hbm = (fetch * fs + write * ws) * 1024
    assert abs(hbm - float(kv["hbm_bytes_per_launch"])) <= 1e-3 * hbm  # scales are printed to 3 decimals
    alg = float(kv["algorithmic_bytes_per_launch"])
    assert alg == 512 * 512 * 1024 * 4 + 1024 * 1024 * 16  # the cube once plus the RGBA image
    assert abs(hbm / alg - float(kv["redundancy"])) < 1e-3


def test_sq_summary_is_consistent():
    kv = bench.read_summary(bench.SQ_FILE)
    samples = 295775536.8125  # nominal samples per frame of the workload (mean of its 16 views)
    per = float(kv["sq_insts_valu_per_launch"]) * 64 / samples
    assert abs(per - float(kv["valu_lane_instr_per_sample"])) < 0.01


def test_several_gpus_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
