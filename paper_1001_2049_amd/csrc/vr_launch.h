// vr_launch.h — host-side entry points into the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr_dev.h"

// Build the bricks of brick layer bz from a linear slab whose first plane is
// z_first.  src_kind: 0 float32 values, 1/2 16-bit codes stored as-is.
hipError_t vr_launch_brick_build(int src_kind, int dst, const void* src, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t z_first, int bz, int Bx, int By,
                                 const uint32_t* slot_of_brick, uint8_t* pool, uint64_t stride,
                                 float* cell_minmax, float sigma, hipStream_t s);

// Per-slot skip masks for one (mode, transfer function, clip) classification.
hipError_t vr_launch_classify(const float* cell_minmax, uint64_t* mask, int nslots, int mode,
                              float clip, float scale, float bias, int n, const int* kpos,
                              hipStream_t s);

// One image, one workgroup per 16x16 tile.
hipError_t vr_launch_render(const DevReq& R, DevCounters* cnt, hipStream_t s);

// Many images in one persistent launch over a (request, tile) work list.
hipError_t vr_launch_batch(const DevReq* reqs, const DevItem* items, int nitems, unsigned* head,
                           DevCounters* cnt, int max_tf_n, int grid, hipStream_t s);
