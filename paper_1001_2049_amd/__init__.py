"""MI355X-native volume renderer for noisy (x, y, frequency) spectral cubes.

Ray casting with trilinear sampling, a 1-D transfer function with a k*sigma
noise clip, front-to-back emission-absorption compositing with early ray
termination, and maximum-intensity projection, in hand-written HIP kernels
for gfx950 behind the C interface in include/vr.h.  ``vr`` is the ctypes
binding of that interface.
"""
from . import vr  # noqa: F401
from .vr import Renderer, VRError  # noqa: F401
