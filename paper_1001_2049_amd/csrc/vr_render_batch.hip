// vr_render_batch.hip — the persistent batched render kernel: many requests
// (cubes, image sizes, modes, storage formats) in one launch.
#include "vr_render.h"

template <int MODE, int DT>
__device__ __forceinline__ void dispatch_interp(const DevReq& R, int tx, int ty, float* tfl,
                                                TileShared& sh, LaneCounts& c) {
    uint8_t* boxes = (uint8_t*)tfl + (MODE == 0 ? 32 * R.tf.n : VR_MIPC_BYTES);
    if (R.interp == 1) render_tile_any<MODE, DT, 1>(R, tx, ty, tfl, boxes, sh, c);
    else render_tile_any<MODE, DT, 0>(R, tx, ty, tfl, boxes, sh, c);
}

template <int MODE>
__device__ __forceinline__ void dispatch_dtype(const DevReq& R, int tx, int ty, float* tfl,
                                               TileShared& sh, LaneCounts& c) {
    if (R.cube.dtype == 1) dispatch_interp<MODE, 1>(R, tx, ty, tfl, sh, c);
    else if (R.cube.dtype == 2) dispatch_interp<MODE, 2>(R, tx, ty, tfl, sh, c);
    else dispatch_interp<MODE, 0>(R, tx, ty, tfl, sh, c);
}

// Persistent grid: each workgroup pulls (request, tile) items until the list is
// exhausted.  Which workgroup renders a tile never changes the tile's pixels.
__global__ __launch_bounds__(VR_WG, VR_WAVES_PER_EU) void k_render_batch(const DevReq* __restrict__ reqs,
                                                        const DevItem* __restrict__ items,
                                                        const int* __restrict__ nitems_p,
                                                        unsigned* head, DevCounters* cnt) {
    extern __shared__ float4 lds4[];
    __shared__ int s_item;
    __shared__ unsigned wgc[5];
    __shared__ TileShared sh;
    float* tfl = (float*)lds4;
    const int nitems = *nitems_p;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
        if (cnt && threadIdx.x < 5) wgc[threadIdx.x] = 0u;
        __syncthreads();
        const int it = s_item;
        if (it >= nitems) break;
        const DevItem item = items[it];
        const DevReq& R = reqs[item.req];
        if (R.mode == 0) tf_stage(R, lds4);
        __syncthreads();
        const int tx = item.tile % R.tiles_x, ty = item.tile / R.tiles_x;
        LaneCounts c = {0u, 0u, 0u, 0u, 0u};
        if (R.mode == 0) dispatch_dtype<0>(R, tx, ty, tfl, sh, c);
        else dispatch_dtype<1>(R, tx, ty, tfl, sh, c);
        if (cnt) flush_counts(c, cnt + item.req, wgc);
        __syncthreads();
    }
}


hipError_t vr_launch_render_batch(const DevReq* reqs, const DevItem* sorted, const int* nitems,
                                  unsigned* head, DevCounters* cnt, size_t lds_bytes, int grid,
                                  hipStream_t s) {
    const hipError_t le = check_lds((const void*)k_render_batch, lds_bytes);
    if (le != hipSuccess) return le;
    hipLaunchKernelGGL(k_render_batch, dim3(grid), dim3(VR_WG), lds_bytes, s, reqs, sorted, nitems,
                       head, cnt);
    return hipGetLastError();
}
