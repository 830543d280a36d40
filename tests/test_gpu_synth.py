"""The GPU evaluation of the synthetic cube generator against the CPU one.

Source terms are tabulated on the host with the C library's exp, so without
noise the two cubes are identical bit for bit; the noise uses the device's
double-precision log/sqrt/sin/cos, so a voxel may differ by one float
rounding step, rarely."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    synth.gpu_lib()  # built by __graft_entry__.build()


@pytest.mark.parametrize("noise", [False, True])
def test_gpu_generator_matches_cpu(noise):
    import torch
    spec = synth.CubeSpec(203, 150, 90, seed=31, noise=noise,
                          sources=synth.SourcePop(40, 3.0, 50.0, True, 1.0, 8.0, 2.0, 40.0))
    cpu = synth.cube(spec)
    out = torch.empty((spec.nz, spec.ny, spec.nx), dtype=torch.float32, device="cuda")
    synth.cube_gpu(spec, out, chunk=16)
    gpu = out.cpu().numpy()
    same = gpu.view(np.uint32) == cpu.view(np.uint32)
    if not noise:
        assert same.all()
    else:
        assert same.mean() > 0.9999
        d = np.abs(gpu[~same].astype(np.float64) - cpu[~same])
        ulp = np.spacing(np.abs(cpu[~same]).astype(np.float32)).astype(np.float64)
        assert (d <= ulp).all()
