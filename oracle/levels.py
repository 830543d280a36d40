"""Coarse levels of the progressive loop — TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module; the renderer never calls it and
shares no code with it.

The paper's thin client turns user interaction into rendering commands (Fig. 1
caption; Sec. 3.1, process step 4) but does not say how a quick first image of
a new view is made.  The reading implemented by the renderer, and written out
here in plain FP64 numpy, is a resolution pyramid of the cube:

* level 0 is the cube itself;
* level L + 1 averages 2 x 2 x 2 blocks of level L: coarse voxel (X, Y, Z)
  is the mean of the level-L voxels with indices {2X, 2X + 1} x {2Y, 2Y + 1}
  x {2Z, 2Z + 1}, an index past the end of an odd-sized axis standing for the
  last voxel (edge clamp, as the sampling of Sec. 2 decision 1 clamps);
* a level-L voxel (X, Y, Z) is centred at fine position 2^L X + (2^L - 1)/2
  (likewise y, z), so the camera is carried into level-L voxel coordinates by
  p -> (p - (2^L - 1)/2) / 2^L (orthographic windows shrink by 2^L, the field
  of view and the up vector are unchanged: the pixel rays are the same lines);
* one level-L voxel length is 2^L fine lengths, so the extinction column of
  the transfer function is multiplied by 2^L (opacity per unit of fine length
  is unchanged); colours, the domain [v0, v1] and the clip are unchanged.

The level-L image is then the ordinary method (the FP64 ray caster) applied
to the level-L cube with that camera and transfer function.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def downsample(vol):
    """One level: the mean of each 2 x 2 x 2 block of ``vol`` ([nz][ny][nx]),
    in float64; an odd axis repeats its last index for the missing half."""
    v = np.asarray(vol, dtype=np.float64)
    nz, ny, nx = v.shape
    iz = [np.minimum(2 * np.arange((nz + 1) // 2) + k, nz - 1) for k in (0, 1)]
    iy = [np.minimum(2 * np.arange((ny + 1) // 2) + k, ny - 1) for k in (0, 1)]
    ix = [np.minimum(2 * np.arange((nx + 1) // 2) + k, nx - 1) for k in (0, 1)]
    acc = np.zeros((len(iz[0]), len(iy[0]), len(ix[0])), dtype=np.float64)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                acc += v[iz[a]][:, iy[b]][:, :, ix[c]]
    return acc / 8.0


def level_volume(vol, L):
    """The level-L cube: ``downsample`` applied L times (level 0: ``vol``)."""
    v = np.asarray(vol, dtype=np.float64)
    for _ in range(L):
        v = downsample(v)
    return v


def level_shape(shape_zyx, L):
    """Axis sizes of the level-L cube: ceil(n / 2) applied L times."""
    s = tuple(int(n) for n in shape_zyx)
    for _ in range(L):
        s = tuple((n + 1) // 2 for n in s)
    return s


def level_camera(cam, L):
    """The camera in level-L voxel coordinates (same type as ``cam``)."""
    k = float(2 ** L)
    off = (k - 1.0) / 2.0
    conv = lambda p: tuple((float(x) - off) / k for x in p)
    return dataclasses.replace(cam, eye=conv(cam.eye), target=conv(cam.target),
                               ortho_w=cam.ortho_w / k, ortho_h=cam.ortho_h / k)


def level_tf(tf, L):
    """Transfer-function rows (r, g, b, kappa) with kappa scaled by 2^L."""
    t = np.array(tf, dtype=np.float64).reshape(-1, 4)
    t[:, 3] *= float(2 ** L)
    return t


def level_size(width, height, L):
    """Image size of level L: ceil(W / 2^L) x ceil(H / 2^L)."""
    return -(-int(width) // 2 ** L), -(-int(height) // 2 ** L)
