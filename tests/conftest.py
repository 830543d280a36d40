import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")


@pytest.fixture(scope="session", autouse=True)
def _c_libraries():
    """The generator and the CPU reference are plain C: build them if absent."""
    import oracle
    import synth
    synth.lib()
    oracle.lib()
    yield


@pytest.fixture(scope="session")
def full_workload():
    """The full-size workload (512x512x1024 float32 cube, generated once per session)."""
    import synth
    wl = synth.full()
    return wl, synth.cube(wl.cube), synth.ramp_tf(256, wl.kappa_max)
