// vr_kernels.hip — HIP kernels for gfx950 (MI355X): upload, classification,
// dispatch order, and the host-side launchers of every kernel.
//
//  k_brick_build  linear cube slab -> 33^3 brick slots (32^3 plus a one-voxel
//                 apron on the + side, edge-clamped), converted to the storage
//                 format, with per-8^3-cell min/max of the stored values.
//                 (The paper partitions the cube into sub-cubes, Sec. 3 process
//                 step 1; here the sub-cube is the unit of memory locality and
//                 of empty-space skipping on one GPU.)
//  k_classify     per brick: a 64-bit mask of the cells where the clipped
//                 transfer function can give non-zero extinction (EA) or where
//                 the maximum reaches the clip (MIP).  Skipped samples would
//                 have contributed exactly nothing, so skipping never changes
//                 the image.
//  k_order_*      per-tile cost estimates and a counting sort that hands the
//                 most expensive tiles out first.
//
// The render kernels themselves live in vr_render.h and are instantiated in
// vr_render_<mode>_<storage>.hip: k_render (one image per launch; a
// 256-thread workgroup renders a 16x16 pixel tile, each 64-lane wave an 8x8
// sub-tile, two workgroups per compute unit) and k_render_batch (a persistent
// grid over the requests of one batch class).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vr_common.h"
#include "vr_dev.h"
#include "vr_launch.h"

// ---------------------------------------------------------------------------
// Brick build: one workgroup per brick of one brick layer (bz fixed)
// ---------------------------------------------------------------------------
#define VR_BRICK_VOX (VR_BRICK_APRON * VR_BRICK_APRON * VR_BRICK_APRON)
#define VR_BB_WG 256

// SRC: 0 float32 values, 1/2 16-bit codes copied as-is.  Every stored element,
// row padding included, holds the edge-clamped value of its global position.
template <int SRC, int DST>
__global__ __launch_bounds__(VR_BB_WG) void k_brick_build(
    const void* __restrict__ src, int64_t nx, int64_t ny, int64_t nz, int64_t z_first, int bz,
    int Bx, int By, uint8_t* __restrict__ pool, uint64_t stride, int xch,
    float* __restrict__ cell_minmax, float sigma, const float* __restrict__ zdiv) {
    __shared__ float vals[VR_BRICK_VOX];
    __shared__ float cmin[VR_CELLS_PER_BRICK], cmax[VR_CELLS_PER_BRICK];
    const int bxi = blockIdx.x % Bx, byi = blockIdx.x / Bx;
    const uint64_t slot = ((uint64_t)bz * By + byi) * Bx + bxi;
    typedef typename Vox<DST>::T DT;
    DT* dst = (DT*)(pool + slot * stride);
    const int64_t x0 = (int64_t)bxi * VR_BRICK, y0 = (int64_t)byi * VR_BRICK,
                  z0 = (int64_t)bz * VR_BRICK;
    constexpr int CV = DST == 0 ? 4 : 8;
    const int nel = VR_SLOT_ZP * VR_SLOT_YG * xch * 8 * CV;
    for (int e = threadIdx.x; e < nel; e += VR_BB_WG) {
        // element e of the slot: chunk e / CV is word (e / CV) % 8 of line e / (8 CV)
        const int sub = e % CV, q = e / CV, w = q & 7, L = q >> 3;
        const int cx = L % xch, yg = (L / xch) % VR_SLOT_YG, zp = L / (xch * VR_SLOT_YG);
        const int lx = cx * CV + sub, ly = yg * 4 + (w & 3), lz = zp * 2 + (w >> 2);
        int64_t gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        gx = gx < nx - 1 ? gx : nx - 1;
        gy = gy < ny - 1 ? gy : ny - 1;
        gz = gz < nz - 1 ? gz : nz - 1;
        const int64_t si = ((gz - z_first) * ny + gy) * nx + gx;
        float dec;
        if (SRC == 0) {
            // stored value: v / sigma, or v / zdiv[z] with per-channel divisors
            const float v = ((const float*)src)[si];
            const float d = zdiv ? zdiv[gz] : sigma;
            if (DST == 0) {
                const float sv = v / d;
                ((float*)dst)[e] = sv;
                dec = sv;
            } else if (DST == 1) {
                const uint16_t c = enc_f16(v / d);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<1>::dec(c);
            } else {
                const uint16_t c = enc_bf16(v / d);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<2>::dec(c);
            }
        } else {
            const uint16_t c = ((const uint16_t*)src)[si];
            ((uint16_t*)dst)[e] = c;
            dec = Vox<DST>::dec(c);
        }
        if (lx < VR_BRICK_APRON && ly < VR_BRICK_APRON && lz < VR_BRICK_APRON)
            vals[(lz * VR_BRICK_APRON + ly) * VR_BRICK_APRON + lx] = dec;
    }
    __syncthreads();
    // 64 cells, 4 threads per cell; cell c covers local [8c, 8c+8] on each axis (9^3)
    {
        const int c = threadIdx.x >> 2, part = threadIdx.x & 3;
        const int cx = c & 3, cy = (c >> 2) & 3, cz = c >> 4;
        float mn = VR_INF, mx = -VR_INF;
        for (int dz = part; dz <= VR_CELL; dz += 4) {
            const int lz = cz * VR_CELL + dz;
            for (int dy = 0; dy <= VR_CELL; ++dy) {
                const int base = (lz * VR_BRICK_APRON + cy * VR_CELL + dy) * VR_BRICK_APRON +
                                 cx * VR_CELL;
                for (int dx = 0; dx <= VR_CELL; ++dx) {
                    const float v = vals[base + dx];
                    mn = fminf(mn, v);
                    mx = fmaxf(mx, v);
                }
            }
        }
        mn = fminf(mn, __shfl_xor(mn, 1));
        mx = fmaxf(mx, __shfl_xor(mx, 1));
        mn = fminf(mn, __shfl_xor(mn, 2));
        mx = fmaxf(mx, __shfl_xor(mx, 2));
        if (part == 0) {
            cmin[c] = mn;
            cmax[c] = mx;
        }
    }
    __syncthreads();
    if (threadIdx.x < VR_CELLS_PER_BRICK) {
        float* cm = cell_minmax + slot * (2 * VR_CELLS_PER_BRICK);
        cm[2 * threadIdx.x] = cmin[threadIdx.x];
        cm[2 * threadIdx.x + 1] = cmax[threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// Skip classification
// ---------------------------------------------------------------------------
// EA: a cell may contribute iff some value v in [max(min, clip), max] maps to a
// table interval with a non-zero kappa at either end.  The value->u map is
// evaluated with exactly the float operations the render kernel uses, so the
// test is conservative for every sample the kernel can produce.
// MIP: a cell may raise the projected maximum above the clip iff max >= clip.
// Output 1: per slot, a 64-bit mask (bit (cz*4 + cy)*4 + cx).
__global__ __launch_bounds__(VR_BB_WG) void k_classify(const float* __restrict__ cell_minmax,
                                                       uint64_t* __restrict__ mask, int nslots,
                                                       int mode, float clip, float scale,
                                                       float bias, int n,
                                                       const int* __restrict__ kpos) {
    const int s = blockIdx.x * VR_BB_WG + threadIdx.x;
    if (s >= nslots) return;
    const float* cm = cell_minmax + (uint64_t)s * (2 * VR_CELLS_PER_BRICK);
    uint64_t m = 0;
    for (int c = 0; c < VR_CELLS_PER_BRICK; ++c) {
        const float mn = cm[2 * c], mx = cm[2 * c + 1];
        bool act;
        if (mode == 1) {
            act = !(mx < clip);
        } else if (mx < clip) {
            act = false;
        } else {
            const float lo = fmaxf(mn, clip);
            const float nm1 = (float)(n - 1), nm2 = (float)(n - 2);
            const float ulo = __builtin_amdgcn_fmed3f(__builtin_fmaf(lo, scale, bias), 0.0f, nm1);
            const float uhi = __builtin_amdgcn_fmed3f(__builtin_fmaf(mx, scale, bias), 0.0f, nm1);
            const int ilo = (int)fminf(floorf(ulo), nm2);
            const int ihi = (int)fminf(floorf(uhi), nm2);
            act = kpos[ihi + 2] - kpos[ilo] > 0;
        }
        m |= (uint64_t)act << c;
    }
    mask[s] = m;
}

// Output 2: the same bits as a global cell grid (4 cells per brick edge, x
// fastest), one thread per 32-bit word (each word holds 8 aligned nibbles).
__global__ __launch_bounds__(VR_BB_WG) void k_cellbits(const uint64_t* __restrict__ mask,
                                                       uint32_t* __restrict__ bits, int nwords,
                                                       int Bx, int By) {
    const int w = blockIdx.x * VR_BB_WG + threadIdx.x;
    if (w >= nwords) return;
    const int Cx = 4 * Bx, Cy = 4 * By;
    uint32_t word = 0;
    for (int q = 0; q < 8; ++q) {
        const int64_t b = (int64_t)w * 32 + 4 * q;
        const int cx = (int)(b % Cx), cy = (int)((b / Cx) % Cy), cz = (int)(b / ((int64_t)Cx * Cy));
        const uint64_t slot = ((uint64_t)(cz >> 2) * By + (cy >> 2)) * Bx + (cx >> 2);
        const uint64_t mk = mask[slot];
        const uint32_t nib = (uint32_t)(mk >> (((cz & 3) * 4 + (cy & 3)) * 4)) & 0xFu;
        word |= nib << (4 * q);
    }
    bits[w] = word;
}

// ---------------------------------------------------------------------------
// Dispatch order: tiles are handed out most expensive first, so that the
// launch does not end waiting on a few long tiles (longest-processing-time
// scheduling).  The cost estimate is the longest lattice among a tile's four
// corner rays and its centre ray; a counting sort over 128 logarithmic cost
// buckets orders the work (the order inside a bucket is arbitrary, and no
// order changes any pixel).
// ---------------------------------------------------------------------------
#define VR_NBUCKET 128

__device__ __forceinline__ int tile_bucket(const DevReq& R, int tile) {
    // plain float, with the hardware reciprocal and reciprocal square root,
    // is enough for an estimate (one workgroup orders a whole image, so this
    // arithmetic is most of the ordering kernel's time)
    const DevCam& C = R.cam;
    const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
    const float xa = (float)(tx * VR_TW) + 0.5f, xb = (float)min(tx * VR_TW + VR_TW, R.W) - 0.5f;
    const float ya = (float)(ty * VR_TH) + 0.5f, yb = (float)min(ty * VR_TH + VR_TH, R.H) - 0.5f;
    const float N[3] = {(float)R.cube.nx, (float)R.cube.ny, (float)R.cube.nz};
    float best = 0.0f;
    for (int k = 0; k < 5; ++k) {
        const float fi = k == 4 ? 0.5f * (xa + xb) : ((k & 1) ? xb : xa);
        const float fj = k == 4 ? 0.5f * (ya + yb) : ((k & 2) ? yb : ya);
        float o[3], d[3], n2 = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const float e = __builtin_fmaf(C.dx[a].hi, fi, __builtin_fmaf(C.dy[a].hi, fj, 0.0f));
            if (C.ortho) {
                o[a] = C.o[a].hi + e;
                d[a] = C.dir[a].hi;
            } else {
                o[a] = C.o[a].hi;
                d[a] = C.base[a].hi + e;
                n2 = __builtin_fmaf(d[a], d[a], n2);
            }
        }
        const float inv = C.ortho ? 1.0f : __builtin_amdgcn_rsqf(n2);
        float t0 = C.ortho ? -VR_INF : 0.0f, t1 = VR_INF;
        for (int a = 0; a < 3; ++a) {
            const float da = d[a] * inv;
            if (da != 0.0f) {
                const float rd = __builtin_amdgcn_rcpf(da);
                const float u = (-0.5f - o[a]) * rd, v = (N[a] - 0.5f - o[a]) * rd;
                t0 = fmaxf(t0, fminf(u, v));
                t1 = fminf(t1, fmaxf(u, v));
            } else if (o[a] < -0.5f || o[a] > N[a] - 0.5f) {
                t1 = -VR_INF;
            }
        }
        best = fmaxf(best, t1 - t0);
    }
    const uint32_t c = (uint32_t)fminf(best / R.step.hi, 1.0e9f) + 16u;
    const int lg = 31 - __builtin_clz(c);  // >= 4
    const int b = 4 * lg + (int)((c >> (lg - 2)) & 3u) - 16;
    return min(max(b, 0), VR_NBUCKET - 1);
}

// hist[0..127]: items per bucket, hist[128..255]: fill cursors
__global__ void k_order_clear(unsigned* hist) {
    if (threadIdx.x < 2 * VR_NBUCKET) hist[threadIdx.x] = 0u;
}

__device__ __forceinline__ void order_offsets(const unsigned* hist, unsigned* off) {
    // off[b] = items in buckets above b (descending cost)
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int b = VR_NBUCKET - 1; b >= 0; --b) {
            off[b] = acc;
            acc += hist[b];
        }
    }
    __syncthreads();
}

__global__ void k_order_count_one(const DevReq R, int n, unsigned* hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&hist[tile_bucket(R, i)], 1u);
}

__global__ void k_order_scatter_one(const DevReq R, int n, unsigned* hist, int* order) {
    __shared__ unsigned off[VR_NBUCKET];
    order_offsets(hist, off);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int b = tile_bucket(R, i);
        order[off[b] + atomicAdd(&hist[VR_NBUCKET + b], 1u)] = i;
    }
}

// Small images: one workgroup buckets every tile, counts in LDS and scatters
// (no global atomics, one launch instead of three).
#define VR_ORDER_FUSED_WG 1024
#define VR_ORDER_FUSED_MAX (16 * VR_ORDER_FUSED_WG)
__global__ __launch_bounds__(VR_ORDER_FUSED_WG) void k_order_fused_one(const DevReq R, int n,
                                                                       int* __restrict__ order) {
    __shared__ unsigned hist[VR_NBUCKET], cur[VR_NBUCKET], off[VR_NBUCKET];
    if (threadIdx.x < VR_NBUCKET) {
        hist[threadIdx.x] = 0u;
        cur[threadIdx.x] = 0u;
    }
    __syncthreads();
    uint8_t bk[VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG];
#pragma unroll
    for (int q = 0; q < VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG; ++q) {
        const int i = threadIdx.x + q * VR_ORDER_FUSED_WG;
        bk[q] = 0;
        if (i < n) {
            const int b = tile_bucket(R, i);
            bk[q] = (uint8_t)b;
            atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    order_offsets(hist, off);
#pragma unroll
    for (int q = 0; q < VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG; ++q) {
        const int i = threadIdx.x + q * VR_ORDER_FUSED_WG;
        if (i < n) order[off[bk[q]] + atomicAdd(&cur[bk[q]], 1u)] = i;
    }
}

// Batches: the work list holds the items of each batch class in one run
// (hdr[2 + k] .. hdr[3 + k] for class k), requests in order inside it.  One
// workgroup per request orders that request's items (found by binary search
// on the request index inside its class's run) most expensive first, in runs
// of up to VR_ORDER_FUSED_MAX items, so each class's persistent launch takes
// its requests one after another, each in longest-first order.
// hdr[1]: requests.
__global__ __launch_bounds__(VR_ORDER_FUSED_WG) void k_order_fused_batch(const DevReq* __restrict__ reqs,
                                                                         const DevItem* __restrict__ items,
                                                                         const int* __restrict__ hdr,
                                                                         DevItem* __restrict__ sorted) {
    __shared__ unsigned hist[VR_NBUCKET], cur[VR_NBUCKET], off[VR_NBUCKET];
    __shared__ int rng[2];
    const int r = blockIdx.x;
    if (r >= hdr[1]) return;
    const DevReq& R = reqs[r];
    const int cls = VR_BATCH_CLASS(R.mode, R.cube.dtype, R.interp);
    if (threadIdx.x < 2) {
        const int key = r + (int)threadIdx.x;  // first item of request r, of request r + 1
        int lo = hdr[2 + cls], hi = hdr[3 + cls];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (items[mid].req < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        rng[threadIdx.x] = lo;
    }
    __syncthreads();
    const int b0 = rng[0], b1 = rng[1];
    for (int c0 = b0; c0 < b1; c0 += VR_ORDER_FUSED_MAX) {
        const int n = min(VR_ORDER_FUSED_MAX, b1 - c0);
        if (threadIdx.x < VR_NBUCKET) {
            hist[threadIdx.x] = 0u;
            cur[threadIdx.x] = 0u;
        }
        __syncthreads();
        uint8_t bk[VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG];
#pragma unroll
        for (int q = 0; q < VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG; ++q) {
            const int i = threadIdx.x + q * VR_ORDER_FUSED_WG;
            bk[q] = 0;
            if (i < n) {
                const int b = tile_bucket(R, items[c0 + i].tile);
                bk[q] = (uint8_t)b;
                atomicAdd(&hist[b], 1u);
            }
        }
        __syncthreads();
        order_offsets(hist, off);
#pragma unroll
        for (int q = 0; q < VR_ORDER_FUSED_MAX / VR_ORDER_FUSED_WG; ++q) {
            const int i = threadIdx.x + q * VR_ORDER_FUSED_WG;
            if (i < n) sorted[c0 + off[bk[q]] + atomicAdd(&cur[bk[q]], 1u)] = items[c0 + i];
        }
        __syncthreads();
    }
}

__global__ void k_reset_head(unsigned* head) {
    if (threadIdx.x < VR_NCLASS && blockIdx.x == 0) head[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <int SRC, int DST>
static hipError_t launch_bb(const void* src, int64_t nx, int64_t ny, int64_t nz, int64_t z_first,
                            int bz, int Bx, int By, uint8_t* pool, uint64_t stride, int xch,
                            float* cell_minmax, float sigma, const float* zdiv, hipStream_t s) {
    hipLaunchKernelGGL((k_brick_build<SRC, DST>), dim3(Bx * By), dim3(VR_BB_WG), 0, s, src, nx,
                       ny, nz, z_first, bz, Bx, By, pool, stride, xch, cell_minmax, sigma, zdiv);
    return hipGetLastError();
}

hipError_t vr_launch_brick_build(int src_kind, int dst, const void* src, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t z_first, int bz, int Bx, int By,
                                 uint8_t* pool, uint64_t stride, int xch, float* cell_minmax,
                                 float sigma, const float* zdiv, hipStream_t s) {
#define VR_BB(S, D)                                                                          \
    if (src_kind == S && dst == D)                                                           \
        return launch_bb<S, D>(src, nx, ny, nz, z_first, bz, Bx, By, pool, stride, xch,      \
                               cell_minmax, sigma, zdiv, s);
    VR_BB(0, 0)
    VR_BB(0, 1)
    VR_BB(0, 2)
    VR_BB(1, 1)
    VR_BB(2, 2)
#undef VR_BB
    return hipErrorInvalidValue;
}

// MIP running-maximum bounds, one per cell in the cell-grid order.  A sample
// in a cell is a trilinear (or nearest) combination of values in [mn, mx]
// (the cell's halo-inclusive range), rounded at each of three lerps; each lerp
// can exceed the larger of its operands by at most about 3 u M (u = 2^-24,
// M = max(|mn|, |mx|)), so every such value lies below mx + 10 u M.  The bound
// adds 2^-19 M (32 u M, still > 30 u M after its own rounding) and a tiny
// absolute term.  A running maximum m >= bound can therefore not be raised by
// any sample of the cell.  Cells entirely below the clip get -inf: under the
// clip floor they never decide the output.
__global__ __launch_bounds__(VR_BB_WG) void k_cellmax(const float* __restrict__ cell_minmax,
                                                      float* __restrict__ cellmax, int64_t ncells,
                                                      int Bx, int By, float clip) {
    const int64_t i = (int64_t)blockIdx.x * VR_BB_WG + threadIdx.x;
    if (i >= ncells) return;
    const int64_t Cx = 4 * (int64_t)Bx, Cy = 4 * (int64_t)By;
    const int cx = (int)(i % Cx), cy = (int)((i / Cx) % Cy);
    const int64_t cz = i / (Cx * Cy);
    const uint64_t slot = ((uint64_t)(cz >> 2) * By + (cy >> 2)) * Bx + (cx >> 2);
    const int c = (int)(((cz & 3) * 4 + (cy & 3)) * 4 + (cx & 3));
    const float mn = cell_minmax[slot * (2 * VR_CELLS_PER_BRICK) + 2 * c];
    const float mx = cell_minmax[slot * (2 * VR_CELLS_PER_BRICK) + 2 * c + 1];
    const float M = fmaxf(fabsf(mn), fabsf(mx));
    cellmax[i] = mx < clip ? -VR_INF : mx + (M * 0x1p-19f + 1e-30f);
}

// Progressive rendering: a coarse level's image enlarged to the full size.
__global__ __launch_bounds__(256) void k_upsample(const float* __restrict__ low, int wl, int hl,
                                                  int ch, float* __restrict__ out, int W, int H,
                                                  int L) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    const int x = (int)(i % W), y = (int)(i / W);
    const int xl = min(x >> L, wl - 1), yl = min(y >> L, hl - 1);
    const float* src = low + ((int64_t)yl * wl + xl) * ch;
    float* dst = out + i * ch;
    if (ch == 4) {
        *(float4*)dst = *(const float4*)src;
    } else {
        dst[0] = src[0];
    }
}

hipError_t vr_launch_upsample(const float* low, int wl, int hl, int ch, float* out, int W, int H,
                              int L, hipStream_t s) {
    const int64_t n = (int64_t)W * H;
    hipLaunchKernelGGL(k_upsample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, low, wl, hl,
                       ch, out, W, H, L);
    return hipGetLastError();
}

hipError_t vr_launch_classify(const float* cell_minmax, uint64_t* mask, uint32_t* cellbits,
                              float* cellmax, int Bx, int By, int Bz, int mode, float clip,
                              float scale, float bias, int n, const int* kpos, hipStream_t s) {
    const int nslots = Bx * By * Bz;
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3((nslots + VR_BB_WG - 1) / VR_BB_WG), dim3(VR_BB_WG), 0, s,
                       cell_minmax, mask, nslots, mode, clip, scale, bias, n, kpos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nwords = vr_cellbits_words(Bx, By, Bz);
    hipLaunchKernelGGL(k_cellbits, dim3((nwords + VR_BB_WG - 1) / VR_BB_WG), dim3(VR_BB_WG), 0, s,
                       (const uint64_t*)mask, cellbits, nwords, Bx, By);
    e = hipGetLastError();
    if (e != hipSuccess || mode != 1 || !cellmax) return e;
    const int64_t ncells = (int64_t)nslots * VR_CELLS_PER_BRICK;
    hipLaunchKernelGGL(k_cellmax, dim3((unsigned)((ncells + VR_BB_WG - 1) / VR_BB_WG)), dim3(VR_BB_WG), 0,
                       s, cell_minmax, cellmax, ncells, Bx, By, clip);
    return hipGetLastError();
}


hipError_t vr_launch_render_0_0(const DevReq&, const int*, DevCounters*, hipStream_t);
hipError_t vr_launch_render_0_1(const DevReq&, const int*, DevCounters*, hipStream_t);
hipError_t vr_launch_render_0_2(const DevReq&, const int*, DevCounters*, hipStream_t);
hipError_t vr_launch_render_1_0(const DevReq&, const int*, DevCounters*, hipStream_t);
hipError_t vr_launch_render_1_1(const DevReq&, const int*, DevCounters*, hipStream_t);
hipError_t vr_launch_render_1_2(const DevReq&, const int*, DevCounters*, hipStream_t);
#define VR_BATCH_LAUNCHER_DECL(MODE, DT)                                                          \
    hipError_t vr_launch_batch_##MODE##_##DT(const DevReq*, const DevItem*, const int*, int, unsigned*, \
                                             DevCounters*, size_t, int, hipStream_t);
VR_BATCH_LAUNCHER_DECL(0, 0)
VR_BATCH_LAUNCHER_DECL(0, 1)
VR_BATCH_LAUNCHER_DECL(0, 2)
VR_BATCH_LAUNCHER_DECL(1, 0)
VR_BATCH_LAUNCHER_DECL(1, 1)
VR_BATCH_LAUNCHER_DECL(1, 2)

hipError_t vr_launch_order(const DevReq& R, int* order, unsigned* hist, hipStream_t s) {
    const int n = R.tiles_x * R.tiles_y;
    if (n <= VR_ORDER_FUSED_MAX) {
        hipLaunchKernelGGL(k_order_fused_one, dim3(1), dim3(VR_ORDER_FUSED_WG), 0, s, R, n, order);
    } else {
        const int ob = (n + 255) / 256;
        hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(2 * VR_NBUCKET), 0, s, hist);
        hipLaunchKernelGGL(k_order_count_one, dim3(ob), dim3(256), 0, s, R, n, hist);
        hipLaunchKernelGGL(k_order_scatter_one, dim3(ob), dim3(256), 0, s, R, n, hist, order);
    }
    return hipGetLastError();
}

hipError_t vr_launch_render(const DevReq& R, int* order, unsigned* hist, DevCounters* cnt,
                            hipStream_t s) {
    const hipError_t e = vr_launch_order(R, order, hist, s);
    if (e != hipSuccess) return e;
    return vr_launch_render_ordered(R, order, cnt, s);
}

hipError_t vr_launch_render_ordered(const DevReq& R, const int* order, DevCounters* cnt,
                                    hipStream_t s) {
    switch (R.mode * 10 + R.cube.dtype) {
        case 0: return vr_launch_render_0_0(R, order, cnt, s);
        case 1: return vr_launch_render_0_1(R, order, cnt, s);
        case 2: return vr_launch_render_0_2(R, order, cnt, s);
        case 10: return vr_launch_render_1_0(R, order, cnt, s);
        case 11: return vr_launch_render_1_1(R, order, cnt, s);
        case 12: return vr_launch_render_1_2(R, order, cnt, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t vr_launch_batch(const DevReq* reqs, const DevItem* items, const int* hdr, int reqs_grid,
                           unsigned class_mask, DevItem* sorted, unsigned* head, DevCounters* cnt,
                           size_t lds_bytes, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_order_fused_batch, dim3(reqs_grid), dim3(VR_ORDER_FUSED_WG), 0, s, reqs, items,
                       hdr, sorted);
    hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, head);
    hipError_t e = hipGetLastError();
    for (int k = 0; k < VR_NCLASS && e == hipSuccess; ++k) {
        if (!(class_mask >> k & 1u)) continue;
        const int mode = k / 6, dt = (k / 2) % 3, interp = k % 2;
        switch (mode * 10 + dt) {
            case 0: e = vr_launch_batch_0_0(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
            case 1: e = vr_launch_batch_0_1(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
            case 2: e = vr_launch_batch_0_2(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
            case 10: e = vr_launch_batch_1_0(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
            case 11: e = vr_launch_batch_1_1(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
            default: e = vr_launch_batch_1_2(reqs, sorted, hdr, interp, head, cnt, lds_bytes, grid, s); break;
        }
    }
    return e;
}
