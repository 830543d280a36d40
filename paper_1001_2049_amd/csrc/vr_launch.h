// vr_launch.h — host-side entry points into the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr_dev.h"

// words of the per-cell skip grid (4 cells per brick edge)
inline int vr_cellbits_words(int Bx, int By, int Bz) {
    const int64_t cells = (int64_t)64 * Bx * By * Bz;
    return (int)((cells + 31) / 32);
}

// LDS bytes reserved ahead of the slab boxes: the transfer function (EA, n
// rows of 32 bytes) or the cell bounds of MIP running-maximum skipping.
inline int vr_lds_reserve(int tf_rows) {
    return 32 * tf_rows > VR_MIPC_BYTES ? 32 * tf_rows : VR_MIPC_BYTES;
}

// LDS bytes of one slab box buffer beside a transfer function of n rows (0: MIP).
// Normally VR_WG_PER_CU workgroups share a compute unit; a transfer function
// too large for that share takes LDS up to the whole unit (fewer workgroups
// then run at once; boxes that do not fit are sampled from the brick pool).
inline int vr_box_bytes(int tf_rows) {
    const int avail = (VR_LDS_CU - VR_LDS_STATIC - vr_lds_reserve(tf_rows)) / 2;
    const int b = (avail / 16) * 16;
    return b < VR_BOX_REF ? b : VR_BOX_REF;
}

// Build the bricks of brick layer bz from a linear slab whose first plane is
// z_first.  src_kind: 0 float32 values, 1/2 16-bit codes stored as-is.
// Float32 values are divided by sigma, or by zdiv[z] (device, one per plane)
// when zdiv is not NULL.
hipError_t vr_launch_brick_build(int src_kind, int dst, const void* src, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t z_first, int bz, int Bx, int By,
                                 uint8_t* pool, uint64_t stride, int xch, float* cell_minmax,
                                 float sigma, const float* zdiv, hipStream_t s);

// Robust noise of `planes` channels (z planes of `plane` floats each, the first
// being plane z_first of the cube) into med/mad/sigma[z] (device arrays).
hipError_t vr_launch_channel_noise(const float* src, int64_t plane, int64_t z_first, int planes,
                                   float* med, float* mad, float* sigma, hipStream_t s);

// Skip masks (per slot) and the per-cell grid for one (mode, transfer function, clip).
// With mode 1 (MIP) and cellmax != NULL also the per-cell bounds of running-
// maximum skipping (see DevCube::cellmax).
hipError_t vr_launch_classify(const float* cell_minmax, uint64_t* mask, uint32_t* cellbits,
                              float* cellmax, int Bx, int By, int Bz, int mode, float clip,
                              float scale, float bias, int n, const int* kpos, hipStream_t s);

// One image, one workgroup per 16x16 tile, dispatched most expensive tile
// first.  order: device scratch of tiles_x * tiles_y ints; hist: 256 words.
hipError_t vr_launch_render(const DevReq& R, int* order, unsigned* hist, DevCounters* cnt,
                            hipStream_t s);
// The two halves of vr_launch_render: the dispatch order of R's tiles into
// `order` (it reads only R's camera, image and cube geometry), and the render
// of R in that order.
hipError_t vr_launch_order(const DevReq& R, int* order, unsigned* hist, hipStream_t s);
hipError_t vr_launch_render_ordered(const DevReq& R, const int* order, DevCounters* cnt,
                                    hipStream_t s);

// Many images in persistent launches over a (request, tile) work list,
// one launch per batch class present (bit k of class_mask: class k, see
// VR_BATCH_CLASS).  The list holds each class's items in one run, requests in
// order inside it; hdr (device, read there so a captured launch serves any
// count): [1] requests, [2 + k] first item of class k, [2 + VR_NCLASS] all
// items.  Each request's tiles are reordered most expensive first into
// `sorted`; reqs_grid: workgroups of the ordering kernel (at least the
// requests); head: VR_NCLASS counters.
hipError_t vr_launch_batch(const DevReq* reqs, const DevItem* items, const int* hdr, int reqs_grid,
                           unsigned class_mask, DevItem* sorted, unsigned* head, DevCounters* cnt,
                           size_t lds_bytes, int grid, hipStream_t s);

// Nearest-neighbour enlargement of a (W >> L) x (H >> L) image (rounded up)
// with `ch` floats per pixel to W x H: output pixel (i, j) takes low pixel
// (i >> L, j >> L).
hipError_t vr_launch_upsample(const float* low, int wl, int hl, int ch, float* out, int W, int H,
                              int L, hipStream_t s);

// Planes [z0, z0 + planes) of the next coarser level of cube c (2x2x2 block
// means of its stored values, edge-clamped on odd axes; the coarser cube is
// ceil(n/2) voxels per axis) into out, float32 [plane][ny2][nx2] (device).
hipError_t vr_launch_mip_down(const DevCube& c, int nx2, int ny2, int z0, int planes, float* out,
                              hipStream_t s);

// Sub-cube partial images (count <= VR_MAX_PARTIALS, sub-cubes in increasing
// plane order along `axis`) combined into one image: EA by front-to-back
// "over" in each pixel's visibility order (the sign of its ray direction on
// the axis, from the camera constants), MIP by maximum and the clip floor.
hipError_t vr_launch_composite(const float* const* partials, int count, int mode, int axis,
                               const DevCam& cam, int W, int H, float* out, hipStream_t s);
