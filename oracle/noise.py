"""Per-channel noise estimation and S/N scaling — TEST INFRASTRUCTURE ONLY.

Reference for the noise-aware variant of the renderer: the paper's attention to
data of low signal-to-noise ratio (abstract; Sec. 2), where the noise level of a
spectral cube varies with frequency.  Each frequency channel (a z plane of the
[z][y][x] cube) gets its own robust noise estimate, and the cube is rendered in
units of that channel's noise, so that a clip at k applies k*sigma(nu) to every
channel (the clip below k*sigma of the renderer, taken per channel).

Definitions (plain, in float64; no blocking, no approximation):
  * median: the lower median, the order statistic of index floor((n-1)/2)
    (0-based) of the channel's n values;
  * MAD: the lower median of |v - median| over the channel (exact in float64:
    both operands are float32 values);
  * sigma = 1.4826 * MAD, the consistent estimator of a Gaussian's standard
    deviation from its median absolute deviation (1/Phi^-1(3/4) = 1.4826...).
A sample of the scaled cube is v / sigma(z); a channel whose MAD is zero is
left unscaled (sigma taken as 1).
"""
from __future__ import annotations

import numpy as np

MAD_TO_SIGMA = 1.4826


def lower_median(x: np.ndarray) -> float:
    """Order statistic of index floor((n-1)/2) of the flattened values."""
    a = np.asarray(x, dtype=np.float64).ravel()
    k = (a.size - 1) // 2
    return float(np.partition(a, k)[k])


def channel_stats(vol: np.ndarray):
    """Per z plane of a [nz][ny][nx] cube: (median, MAD, sigma) as float64 arrays."""
    v = np.asarray(vol)
    nz = v.shape[0]
    med = np.empty(nz)
    mad = np.empty(nz)
    for z in range(nz):
        plane = v[z].astype(np.float64).ravel()
        med[z] = lower_median(plane)
        mad[z] = lower_median(np.abs(plane - med[z]))
    sigma = MAD_TO_SIGMA * mad
    return med, mad, sigma


def scale_divisors(sigma: np.ndarray) -> np.ndarray:
    """Divisor per channel: sigma, or 1 where the MAD vanished."""
    s = np.asarray(sigma, dtype=np.float64)
    return np.where(s > 0.0, s, 1.0)


def scaled_cube(vol: np.ndarray, divisors: np.ndarray) -> np.ndarray:
    """The cube in units of each channel's noise (float64)."""
    v = np.asarray(vol, dtype=np.float64)
    return v / np.asarray(divisors, dtype=np.float64)[:, None, None]
