// vr_mip.hip — the resolution pyramid behind the progressive loop's coarse
// levels.
//
//  k_mip_down  planes [z0, z0 + planes) of the next coarser level of a cube:
//              voxel (X, Y, Z) is the mean of the cube's stored values at
//              {2X, 2X+1} x {2Y, 2Y+1} x {2Z, 2Z+1}, an index past the end of
//              an odd axis reading that axis's last voxel.  The result goes to
//              a linear float32 [plane][y][x] slab, from which the brick build
//              makes the coarser cube's slots and cell statistics, one brick
//              layer at a time.  Memory-bound and run once per cube and level.
#include <algorithm>

#include "vr_render.h"

#define VR_MIP_WG 256

template <int DT>
__global__ __launch_bounds__(VR_MIP_WG) void k_mip_down(const DevCube c, int nx2, int ny2, int z0,
                                                        int planes, float* __restrict__ out) {
    const int64_t n = (int64_t)nx2 * ny2 * planes;
    for (int64_t i = (int64_t)blockIdx.x * VR_MIP_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VR_MIP_WG) {
        const int X = (int)(i % nx2);
        const int64_t r = i / nx2;
        const int Y = (int)(r % ny2);
        const int Z = z0 + (int)(r / ny2);
        const int xa = 2 * X, xb = min(2 * X + 1, c.nx - 1);
        const int ya = 2 * Y, yb = min(2 * Y + 1, c.ny - 1);
        const int za = 2 * Z, zb = min(2 * Z + 1, c.nz - 1);
        auto v = [&](int x, int y, int z) { return pool_value<DT, 0>(c, x, y, z, 0.0f, 0.0f, 0.0f); };
        const float lo = (v(xa, ya, za) + v(xb, ya, za)) + (v(xa, yb, za) + v(xb, yb, za));
        const float hi = (v(xa, ya, zb) + v(xb, ya, zb)) + (v(xa, yb, zb) + v(xb, yb, zb));
        out[i] = (lo + hi) * 0.125f;
    }
}

hipError_t vr_launch_mip_down(const DevCube& c, int nx2, int ny2, int z0, int planes, float* out,
                              hipStream_t s) {
    const int64_t n = (int64_t)nx2 * ny2 * planes;
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + VR_MIP_WG - 1) / VR_MIP_WG, 16384);
    switch (c.dtype) {
        case 0: k_mip_down<0><<<grid, VR_MIP_WG, 0, s>>>(c, nx2, ny2, z0, planes, out); break;
        case 1: k_mip_down<1><<<grid, VR_MIP_WG, 0, s>>>(c, nx2, ny2, z0, planes, out); break;
        default: k_mip_down<2><<<grid, VR_MIP_WG, 0, s>>>(c, nx2, ny2, z0, planes, out); break;
    }
    return hipGetLastError();
}
