// vr_kernels.hip — HIP kernels for gfx950 (MI355X).
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
//  k_render       one ray per pixel (Sec. 2 design decision 1, Sec. 3 process
//                 step 3); a 64-lane wave owns an 8x8 pixel tile and a
//                 256-thread workgroup a 16x16 tile.  Samples are trilinear
//                 (or nearest) on a per-ray lattice of midpoints; EA
//                 compositing front to back with early termination, or MIP.
//  k_render_batch the same per-tile work pulled from a work list by a
//                 persistent grid: many requests (cubes, image sizes, modes)
//                 in one launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vr_dev.h"
#include "vr_launch.h"

#define VR_INF __builtin_huge_valf()


#define VR_LOG2E 1.4426950408889634f

// ---------------------------------------------------------------------------
// Storage formats
// ---------------------------------------------------------------------------
template <int DT>
struct Vox;
template <>
struct Vox<0> {
    typedef float T;
    static __device__ __forceinline__ float dec(float v) { return v; }
};
template <>
struct Vox<1> {
    typedef uint16_t T;
    static __device__ __forceinline__ float dec(uint16_t v) {
        return (float)__builtin_bit_cast(_Float16, v);
    }
};
template <>
struct Vox<2> {
    typedef uint16_t T;
    static __device__ __forceinline__ float dec(uint16_t v) {
        return __builtin_bit_cast(float, (uint32_t)v << 16);
    }
};

// round-to-nearest-even float -> bfloat16 code (finite inputs)
__device__ __forceinline__ uint16_t enc_bf16(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t enc_f16(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}


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
    int Bx, int By, uint8_t* __restrict__ pool, uint64_t stride, int row,
    float* __restrict__ cell_minmax, float sigma) {
    __shared__ float vals[VR_BRICK_VOX];
    __shared__ float cmin[VR_CELLS_PER_BRICK], cmax[VR_CELLS_PER_BRICK];
    const int bxi = blockIdx.x % Bx, byi = blockIdx.x / Bx;
    const uint64_t slot = ((uint64_t)bz * By + byi) * Bx + bxi;
    typedef typename Vox<DST>::T DT;
    DT* dst = (DT*)(pool + slot * stride);
    const int64_t x0 = (int64_t)bxi * VR_BRICK, y0 = (int64_t)byi * VR_BRICK,
                  z0 = (int64_t)bz * VR_BRICK;
    const int nel = VR_BRICK_APRON * VR_BRICK_APRON * row;
    for (int e = threadIdx.x; e < nel; e += VR_BB_WG) {
        const int lx = e % row, ly = (e / row) % VR_BRICK_APRON, lz = e / (row * VR_BRICK_APRON);
        int64_t gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        gx = gx < nx - 1 ? gx : nx - 1;
        gy = gy < ny - 1 ? gy : ny - 1;
        gz = gz < nz - 1 ? gz : nz - 1;
        const int64_t si = ((gz - z_first) * ny + gy) * nx + gx;
        float dec;
        if (SRC == 0) {
            const float v = ((const float*)src)[si];
            if (DST == 0) {
                const float sv = v / sigma;
                ((float*)dst)[e] = sv;
                dec = sv;
            } else if (DST == 1) {
                const uint16_t c = enc_f16(v / sigma);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<1>::dec(c);
            } else {
                const uint16_t c = enc_bf16(v / sigma);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<2>::dec(c);
            }
        } else {
            const uint16_t c = ((const uint16_t*)src)[si];
            ((uint16_t*)dst)[e] = c;
            dec = Vox<DST>::dec(c);
        }
        if (lx < VR_BRICK_APRON) vals[(lz * VR_BRICK_APRON + ly) * VR_BRICK_APRON + lx] = dec;
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
// Rendering: shared pieces
// ---------------------------------------------------------------------------
// Workgroups are dealt to the 8 XCDs round-robin; remap so that each XCD gets
// a contiguous band of tiles (neighbouring rays then share that XCD's L2).
__device__ __forceinline__ int xcd_swizzle(int g, int num) {
    const int x = g & 7, k = g >> 3, per = num >> 3, rem = num & 7;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

struct LaneCounts {
    unsigned nominal, exec, hit, ert, skipped;
};

// One ray: origin/direction and chord in float-float, the sample lattice.
struct Ray {
    ff o[3], d[3];
    ff tin;
    int n;                 // lattice samples; 0 when the ray misses the cube
    float last_adj;        // the last segment's midpoint, in lattice steps before a full step's
    float c_full, c_last;  // -len * log2(e) of full and last segments
    float dd[3];           // step * direction
};

// Ray through pixel-centre coordinates (fi, fj).  Both camera kinds produce
// scalar values that are stored once, after the branch (stores sunk out of
// the two branches would otherwise select between stack addresses).
__device__ __forceinline__ void ray_dir(const DevCam& cam, float fi, float fj, ff o[3], ff d[3]) {
    ff o0, o1, o2, d0, d1, d2;
    if (cam.ortho) {
        o0 = ff_add(ff_add(cam.o[0], ff_mul_f(cam.dx[0], fi)), ff_mul_f(cam.dy[0], fj));
        o1 = ff_add(ff_add(cam.o[1], ff_mul_f(cam.dx[1], fi)), ff_mul_f(cam.dy[1], fj));
        o2 = ff_add(ff_add(cam.o[2], ff_mul_f(cam.dx[2], fi)), ff_mul_f(cam.dy[2], fj));
        d0 = cam.dir[0];
        d1 = cam.dir[1];
        d2 = cam.dir[2];
    } else {
        const ff e0 = ff_add(ff_add(cam.base[0], ff_mul_f(cam.dx[0], fi)), ff_mul_f(cam.dy[0], fj));
        const ff e1 = ff_add(ff_add(cam.base[1], ff_mul_f(cam.dx[1], fi)), ff_mul_f(cam.dy[1], fj));
        const ff e2 = ff_add(ff_add(cam.base[2], ff_mul_f(cam.dx[2], fi)), ff_mul_f(cam.dy[2], fj));
        const ff n2 = ff_add(ff_add(ff_mul(e0, e0), ff_mul(e1, e1)), ff_mul(e2, e2));
        const ff inv = ff_div(ff_make(1.0f), ff_sqrt(n2));
        d0 = ff_mul(e0, inv);
        d1 = ff_mul(e1, inv);
        d2 = ff_mul(e2, inv);
        o0 = cam.o[0];
        o1 = cam.o[1];
        o2 = cam.o[2];
    }
    o[0] = o0;
    o[1] = o1;
    o[2] = o2;
    d[0] = d0;
    d[1] = d1;
    d[2] = d2;
}

// Camera ray of pixel (px, py), its chord through [-1/2, N-1/2]^3 and the
// lattice of n = ceil(L/step) segments sampled at their midpoints.
__device__ __forceinline__ void ray_setup(const DevReq& R, int px, int py, Ray& ray) {
    ray_dir(R.cam, (float)px + 0.5f, (float)py + 0.5f, ray.o, ray.d);
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    ff tin = ff_make(R.cam.ortho ? -VR_INF : 0.0f);
    ff tout = ff_make(VR_INF);
    bool hit = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hib = (float)N[a] - 0.5f;
        if (ray.d[a].hi != 0.0f) {
            const ff t0 = ff_div(ff_sub(ff_make(-0.5f), ray.o[a]), ray.d[a]);
            const ff t1 = ff_div(ff_sub(ff_make(hib), ray.o[a]), ray.d[a]);
            tin = ff_max(tin, ff_min(t0, t1));
            tout = ff_min(tout, ff_max(t0, t1));
        } else if (ff_lt(ray.o[a], ff_make(-0.5f)) || ff_lt(ff_make(hib), ray.o[a])) {
            hit = false;
        }
    }
    hit = hit && ff_lt(tin, tout);
    if (!hit) {
        ray.n = 0;
        return;
    }
    const ff L = ff_sub(tout, tin);
    const ff rr = ff_div(L, R.step);
    float nf = ceilf(rr.hi);
    if (nf == rr.hi && rr.lo > 0.0f) nf += 1.0f;
    ray.n = nf < 1.0f ? 1 : (int)nf;
    ray.tin = tin;
    const float stepf = ff_to_f(R.step);
    float len_last = ff_to_f(ff_sub(L, ff_mul_f(R.step, (float)(ray.n - 1))));
    len_last = fmaxf(len_last, 0.0f);
    ray.last_adj = 0.5f * (len_last / stepf - 1.0f);
    ray.c_full = -stepf * VR_LOG2E;
    ray.c_last = -len_last * VR_LOG2E;
#pragma unroll
    for (int a = 0; a < 3; ++a) ray.dd[a] = ff_to_f(ff_mul(ray.d[a], R.step));
}

// Parameter t of lattice sample k.
__device__ __forceinline__ ff sample_t(const DevReq& R, const Ray& ray, int k) {
    ff t = ff_add(ray.tin, ff_mul_f(R.step, (float)k + 0.5f));
    if (k == ray.n - 1) t = ff_add(t, ff_make(ray.last_adj * ff_to_f(R.step)));
    return t;
}

// Stored value of global voxel (gx, gy, gz) in the brick pool; its +x/+y/+z
// neighbours are in the same slot thanks to the apron.
template <int DT>
__device__ __forceinline__ const typename Vox<DT>::T* pool_ptr(const DevCube& c, int gx, int gy,
                                                               int gz) {
    const uint64_t slot = ((uint64_t)(gz >> 5) * c.by + (gy >> 5)) * c.bx + (gx >> 5);
    const int idx = ((gz & 31) * VR_BRICK_APRON + (gy & 31)) * c.row + (gx & 31);
    return (const typename Vox<DT>::T*)(c.pool + slot * c.stride) + idx;
}

// Trilinear interpolation of the 8 corners (x, then y, then z).
__device__ __forceinline__ float trilerp(float c000, float c100, float c010, float c110, float c001,
                                         float c101, float c011, float c111, float w0, float w1,
                                         float w2) {
    const float x00 = __builtin_fmaf(w0, c100 - c000, c000);
    const float x10 = __builtin_fmaf(w0, c110 - c010, c010);
    const float x01 = __builtin_fmaf(w0, c101 - c001, c001);
    const float x11 = __builtin_fmaf(w0, c111 - c011, c011);
    const float y0 = __builtin_fmaf(w1, x10 - x00, x00);
    const float y1 = __builtin_fmaf(w1, x11 - x01, x01);
    return __builtin_fmaf(w2, y1 - y0, y0);
}

// Value at a corner-0 pointer with strides (1, sy, sz) in elements.
template <int DT, int INTERP, typename P>
__device__ __forceinline__ float interp_at(P bp, int sy, int sz, float w0, float w1, float w2) {
    if (INTERP == 1) {
        return trilerp(Vox<DT>::dec(bp[0]), Vox<DT>::dec(bp[1]), Vox<DT>::dec(bp[sy]),
                       Vox<DT>::dec(bp[sy + 1]), Vox<DT>::dec(bp[sz]), Vox<DT>::dec(bp[sz + 1]),
                       Vox<DT>::dec(bp[sz + sy]), Vox<DT>::dec(bp[sz + sy + 1]), w0, w1, w2);
    }
    return Vox<DT>::dec(bp[0]);
}

// Accumulation state of one ray.
struct Accum {
    float C0, C1, C2, T, m;
};

// Classify sample value v and composite it front to back; returns true when
// the ray becomes opaque enough to stop.
__device__ __forceinline__ bool composite(const DevReq& R, const float* __restrict__ tfl, float v,
                                          bool last, const Ray& ray, Accum& acc) {
    float u = __builtin_fmaf(v, R.tf.scale, R.tf.bias);
    u = __builtin_amdgcn_fmed3f(u, 0.0f, (float)(R.tf.n - 1));
    const float fl = fminf(floorf(u), (float)(R.tf.n - 2));
    const float g = u - fl;
    const float4* row = (const float4*)(tfl + 8 * (int)fl);
    const float4 r0 = row[0], dr = row[1];
    float kap = __builtin_fmaf(g, dr.w, r0.w);
    kap = v < R.tf.clip ? 0.0f : kap;
    // emission-absorption over the segment: alpha = 1 - exp(-kappa len)
    const float ex = __builtin_amdgcn_exp2f(kap * (last ? ray.c_last : ray.c_full));
    const float wgt = acc.T * (1.0f - ex);
    acc.C0 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.x, r0.x), acc.C0);
    acc.C1 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.y, r0.y), acc.C1);
    acc.C2 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.z, r0.z), acc.C2);
    acc.T *= ex;
    return acc.T <= R.ert_T;
}

template <int MODE>
__device__ __forceinline__ void store_pixel(const DevReq& R, int px, int py, bool hit,
                                            const Accum& acc) {
    const int64_t pix = (int64_t)py * R.W + px;
    if (MODE == 0) {
        *(float4*)(R.out + 4 * pix) =
            hit ? make_float4(acc.C0, acc.C1, acc.C2, 1.0f - acc.T) : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        R.out[pix] = hit ? ((acc.m >= R.tf.clip) ? acc.m * R.out_scale : 0.0f) : -VR_INF;
    }
}

__device__ __forceinline__ void tile_pixel(const DevReq& R, int tx, int ty, int& px, int& py) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    px = tx * VR_TW + (wave & 3) * 8 + (lane & 7);
    py = ty * VR_TH + (wave >> 2) * 8 + (lane >> 3);
}

// ---------------------------------------------------------------------------
// Per-ray brick walker (used when the rays of a tile diverge too much to
// share a slab axis, e.g. tiny images with a wide field of view).  Positions
// are anchored in float-float at every brick entry and advanced in float in
// brick-local coordinates; empty 8^3 cells are jumped over.
// ---------------------------------------------------------------------------
template <int MODE, int DT, int INTERP>
__device__ __forceinline__ void render_lane_direct(const DevReq& R, const int px, const int py,
                                                   const float* __restrict__ tfl, LaneCounts& cnt) {
    typedef typename Vox<DT>::T VT;
    Ray ray;
    ray_setup(R, px, py, ray);
    const int n = ray.n;
    Accum acc = {0.0f, 0.0f, 0.0f, 1.0f, -VR_INF};
    if (n == 0) {
        store_pixel<MODE>(R, px, py, false, acc);
        return;
    }
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    const int B[3] = {R.cube.bx, R.cube.by, R.cube.bz};
    const int sy = R.cube.row, sz = VR_BRICK_APRON * R.cube.row;
    float inv_dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) inv_dd[a] = ray.dd[a] != 0.0f ? 1.0f / ray.dd[a] : 0.0f;
    const float shift = INTERP == 0 ? 0.5f : 0.0f;
    int k0 = 0, m = 0, j = 0;
    float A[3] = {0.0f, 0.0f, 0.0f}, hb[3] = {0.0f, 0.0f, 0.0f};
    const uint8_t* base = nullptr;
    uint64_t mask = 0;
    unsigned nexec = 0, nskip = 0;
    bool stopped = false;
    while (true) {
        if (j >= m) {
            k0 += m;
            if (k0 >= n) break;
            const ff t = sample_t(R, ray, k0);
            int b[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const ff P = ff_add(ray.o[a], ff_mul(t, ray.d[a]));
                int bb = (int)floorf(P.hi * (1.0f / VR_BRICK));
                bb = bb < 0 ? 0 : (bb > B[a] - 1 ? B[a] - 1 : bb);
                b[a] = bb;
                A[a] = ff_to_f(ff_add(P, ff_make(-(float)(VR_BRICK * bb))));
                hb[a] = fminf(31.999998f, (float)(N[a] - 1 - VR_BRICK * bb));
            }
            float s = VR_INF;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (ray.dd[a] > 0.0f && b[a] < B[a] - 1)
                    s = fminf(s, ((float)VR_BRICK - A[a]) * inv_dd[a]);
                if (ray.dd[a] < 0.0f && b[a] > 0) s = fminf(s, (-A[a]) * inv_dd[a]);
            }
            const int rem = n - k0;
            m = s >= (float)rem ? rem : max(1, (int)ceilf(s));
            j = 0;
            const uint64_t slot = ((uint64_t)b[2] * B[1] + b[1]) * B[0] + b[0];
            base = R.cube.pool + slot * R.cube.stride;
            mask = R.use_skip ? R.cube.mask[slot] : ~0ull;
            if (mask == 0) {
                nskip += m;
                j = m;
                continue;
            }
        }
        const bool last = (k0 + j == n - 1);
        const float jf = (float)j + ((last && j > 0) ? ray.last_adj : 0.0f);
        const float p0 = __builtin_fmaf(jf, ray.dd[0], A[0]);
        const float p1 = __builtin_fmaf(jf, ray.dd[1], A[1]);
        const float p2 = __builtin_fmaf(jf, ray.dd[2], A[2]);
        const float q0 = __builtin_amdgcn_fmed3f(p0, 0.0f, hb[0]);
        const float q1 = __builtin_amdgcn_fmed3f(p1, 0.0f, hb[1]);
        const float q2 = __builtin_amdgcn_fmed3f(p2, 0.0f, hb[2]);
        int i0, i1, i2, cell;
        float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
        if (INTERP == 1) {
            const float f0 = floorf(q0), f1 = floorf(q1), f2 = floorf(q2);
            w0 = q0 - f0;
            w1 = q1 - f1;
            w2 = q2 - f2;
            i0 = (int)f0;
            i1 = (int)f1;
            i2 = (int)f2;
            cell = (i0 >> 3) | ((i1 >> 3) << 2) | ((i2 >> 3) << 4);
        } else {
            i0 = (int)floorf(q0 + 0.5f);
            i1 = (int)floorf(q1 + 0.5f);
            i2 = (int)floorf(q2 + 0.5f);
            cell = (min(i0, 31) >> 3) | ((min(i1, 31) >> 3) << 2) | ((min(i2, 31) >> 3) << 4);
        }
        if (!((mask >> cell) & 1ull)) {
            // jump to the first sample past this cell, pulling the cell's faces in by
            // 1e-4 voxel so rounding can never skip a sample of the next cell
            const int c3[3] = {cell & 3, (cell >> 2) & 3, cell >> 4};
            const float pw[3] = {p0 + shift, p1 + shift, p2 + shift};
            float s = VR_INF;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (ray.dd[a] > 0.0f)
                    s = fminf(s, ((float)(VR_CELL * (c3[a] + 1)) - 1e-4f - pw[a]) * inv_dd[a]);
                else if (ray.dd[a] < 0.0f)
                    s = fminf(s, ((float)(VR_CELL * c3[a]) + 1e-4f - pw[a]) * inv_dd[a]);
            }
            const int jump = s >= 1.0e6f ? (1 << 20) : max(1, (int)ceilf(s));
            nskip += min(jump, m - j);
            j += jump;
            continue;
        }
        const int idx = (i2 * VR_BRICK_APRON + i1) * sy + i0;
        const float v = interp_at<DT, INTERP>((const VT*)base + idx, sy, sz, w0, w1, w2);
        ++nexec;
        ++j;
        if (MODE == 1) {
            acc.m = fmaxf(acc.m, v);
            continue;
        }
        if (composite(R, tfl, v, last, ray, acc)) {
            stopped = true;
            break;
        }
    }
    store_pixel<MODE>(R, px, py, true, acc);
    cnt.nominal += (unsigned)n;
    cnt.exec += nexec;
    cnt.hit += 1u;
    cnt.ert += stopped ? 1u : 0u;
    cnt.skipped += nskip;
}

// ---------------------------------------------------------------------------
// Slab-staged tile renderer (the main path).
//
// A 512-thread workgroup owns a 32x16 pixel tile and marches all its rays in
// lock-step through slabs S voxels thick along the major axis M of the tile's
// view direction, front to back.  For each slab it reduces the range of voxel
// indices its samples touch (a box), tests the box's 8^3 cells against the
// skip grid, copies the box into LDS with 16-byte global->LDS DMA, and every
// lane then interpolates its ray's samples in that slab from LDS.  Two box
// buffers and a two-slab lookahead let the copy of slab k+1 and the skip-grid
// reads of slab k+2 run while slab k is sampled; each slab costs one barrier.
// A box larger than its buffer is sampled straight from the brick pool with
// the same arithmetic, so the image never depends on staging decisions.
// ---------------------------------------------------------------------------
#define VR_RING 5
#define VR_BIG 0x3fffffff

struct SlabDesc {
    int bmin[3], bmax[3];  // sample floor range, relative to the slab origin
    int any;               // some cell of the box may contribute
    int pad;
};

struct TileShared {
    int red[12];           // tile-start reductions
    SlabDesc d[VR_RING];   // slab descriptors, ring indexed by slab % VR_RING
    int alive[3];          // rays still marching after slab k, ring by k % 3
};

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <int INTERP>
__device__ __forceinline__ void floor_idx(const float p[3], const float lo[3], const float hi[3],
                                          int i[3], float w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = __builtin_amdgcn_fmed3f(p[a], lo[a], hi[a]);
        if (INTERP == 1) {
            const float f = floorf(q);
            w[a] = q - f;
            i[a] = (int)f;
        } else {
            w[a] = 0.0f;
            i[a] = (int)floorf(q + 0.5f);
        }
    }
}

// exact i / d for 0 <= i < 2^22 and 0 < d < 2^22 via a float reciprocal
__device__ __forceinline__ int div_small(int i, int d, float inv_d) {
    int q = (int)((float)i * inv_d);
    q -= q * d > i ? 1 : 0;
    q += (q + 1) * d <= i ? 1 : 0;
    return q;
}

// Geometry of slab k that every lane derives identically.
template <int M>
struct SlabGeo {
    int B0[3];     // integer origin of the slab's local coordinates
    float zexit;   // plane the rays cross when leaving the slab
};

template <int M>
__device__ __forceinline__ SlabGeo<M> slab_geo(int k, int Z0, int S, int sgn, const float* rf,
                                               const float* cf) {
    constexpr int A1 = (M + 1) % 3, A2 = (M + 2) % 3;
    SlabGeo<M> g;
    const int zlow = sgn > 0 ? Z0 + S * k : Z0 - S * (k + 1);
    g.zexit = (float)(sgn > 0 ? zlow + S : zlow);
    const float zmid = (float)zlow + 0.5f * (float)S;
    g.B0[M] = zlow;
    g.B0[A1] = (int)floorf(__builtin_fmaf(zmid, rf[A1], cf[A1]));
    g.B0[A2] = (int)floorf(__builtin_fmaf(zmid, rf[A2], cf[A2]));
    return g;
}

// Samples [k0, k1) of one ray in a slab with origin B0: local anchor and clamp bounds.
__device__ __forceinline__ void slab_anchor(const DevReq& R, const Ray& ray, int k0,
                                            const int B0[3], float A[3], float lo[3], float hi[3]) {
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    const ff t0 = sample_t(R, ray, k0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        A[a] = ff_to_f(ff_add(ff_add(ray.o[a], ff_mul(t0, ray.d[a])), ff_make(-(float)B0[a])));
        lo[a] = (float)(-B0[a]);
        hi[a] = (float)(N[a] - 1 - B0[a]);
    }
}

// Derived box geometry of a reduced slab descriptor.
struct BoxGeo {
    int blo[3], bdim[3], g0[3];
    int xa, nc, pitch, elems;
    bool empty;
};

template <int DT, int INTERP>
__device__ __forceinline__ BoxGeo box_geo(const SlabDesc& d, const int B0[3]) {
    constexpr int CV = DT == 0 ? 4 : 8;
    BoxGeo b;
    b.empty = d.bmin[0] > d.bmax[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b.blo[a] = d.bmin[a];
        b.bdim[a] = d.bmax[a] - d.bmin[a] + 1 + (INTERP == 1 ? 1 : 0);
        b.g0[a] = B0[a] + b.blo[a];
    }
    b.xa = b.g0[0] & ~(CV - 1);
    b.nc = (b.g0[0] + b.bdim[0] - 1 - b.xa) / CV + 1;
    b.pitch = b.nc * CV;
    b.elems = b.empty ? 0 : b.pitch * b.bdim[1] * b.bdim[2];
    return b;
}

template <int MODE, int DT, int INTERP, int M>
__device__ __forceinline__ bool tile_march(const DevReq& R, const Ray& ray, const int px,
                                           const int py, const bool inimg, const ff* oc,
                                           const ff* dc, const int sgn,
                                           const float* __restrict__ tfl, uint8_t* __restrict__ boxes,
                                           TileShared& sh, LaneCounts& cnt) {
    typedef typename Vox<DT>::T VT;
    constexpr int A1 = (M + 1) % 3, A2 = (M + 2) % 3;
    constexpr int ELEM = DT == 0 ? 4 : 2;
    constexpr int CV = 16 / ELEM;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    const int cap = R.box_bytes / ELEM;
    const bool act = ray.n > 0;

    // ---- tile-wide set-up: common axis, slab range, lateral spread -------------
    // reference ray (tile centre): position on plane z is cf + z * rf
    float rf[3], cf[3];
    {
        const float ocm = ff_to_f(oc[M]), dcm = dc[M].hi;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rf[a] = a == M ? 1.0f : dc[a].hi / dcm;
            cf[a] = a == M ? 0.0f : ff_to_f(oc[a]) - ocm * rf[a];
        }
    }
    int zf = VR_BIG, zl = VR_BIG, dlo1 = VR_BIG, dhi1 = -VR_BIG, dlo2 = VR_BIG, dhi2 = -VR_BIG;
    int sl1 = 0, sl2 = 0, okl = 1;
    if (act) {
        const ff t0 = sample_t(R, ray, 0), t1 = sample_t(R, ray, ray.n - 1);
        float pf[3], pl[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pf[a] = ff_to_f(ff_add(ray.o[a], ff_mul(t0, ray.d[a])));
            pl[a] = ff_to_f(ff_add(ray.o[a], ff_mul(t1, ray.d[a])));
        }
        okl = (float)sgn * ray.d[M].hi >= 0.25f;
        const float hm = (float)(N[M] - 1);
        zf = (int)floorf(fminf(fmaxf(pf[M], 0.0f), hm));
        zl = (int)floorf(fminf(fmaxf(pl[M], 0.0f), hm));
        const float e1f = pf[A1] - __builtin_fmaf(pf[M], rf[A1], cf[A1]);
        const float e1l = pl[A1] - __builtin_fmaf(pl[M], rf[A1], cf[A1]);
        const float e2f = pf[A2] - __builtin_fmaf(pf[M], rf[A2], cf[A2]);
        const float e2l = pl[A2] - __builtin_fmaf(pl[M], rf[A2], cf[A2]);
        dlo1 = (int)floorf(fminf(e1f, e1l));
        dhi1 = (int)ceilf(fmaxf(e1f, e1l));
        dlo2 = (int)floorf(fminf(e2f, e2l));
        dhi2 = (int)ceilf(fmaxf(e2f, e2l));
        const float inv = 1.0f / fabsf(ray.d[M].hi);
        sl1 = (int)ceilf(fabsf(ray.d[A1].hi) * inv * 1024.0f);
        sl2 = (int)ceilf(fabsf(ray.d[A2].hi) * inv * 1024.0f);
    }
    {
        const int zfn = wave_min(act ? zf : VR_BIG), zfx = wave_max(act ? zf : -VR_BIG);
        const int zln = wave_min(act ? zl : VR_BIG), zlx = wave_max(act ? zl : -VR_BIG);
        const int a = wave_min(dlo1), b = wave_max(dhi1), c = wave_min(dlo2), d = wave_max(dhi2);
        const int e = wave_max(sl1), f = wave_max(sl2);
        const bool okw = __ballot(!okl) == 0ull;
        if (lane == 0) {
            atomicMin(&sh.red[0], zfn);
            atomicMax(&sh.red[1], zfx);
            atomicMin(&sh.red[2], zln);
            atomicMax(&sh.red[3], zlx);
            atomicMin(&sh.red[4], a);
            atomicMax(&sh.red[5], b);
            atomicMin(&sh.red[6], c);
            atomicMax(&sh.red[7], d);
            atomicMax(&sh.red[8], e);
            atomicMax(&sh.red[9], f);
            if (!okw) atomicAnd(&sh.red[10], 0);
        }
    }
    __syncthreads();
    if (!sh.red[10]) return false;
    const bool any_ray = sh.red[0] != VR_BIG;
    // slab thickness: the thickest whose worst-case box fits one buffer
    int S = 0;
    if (any_ray) {
        const int sp1 = sh.red[5] - sh.red[4] + 1, sp2 = sh.red[7] - sh.red[6] + 1;
        const float s1 = (float)sh.red[8] * (1.0f / 1024.0f), s2 = (float)sh.red[9] * (1.0f / 1024.0f);
        for (int cand = 16; cand >= 1; cand >>= 1) {
            int ext[3];
            ext[M] = cand + 3;
            ext[A1] = sp1 + (int)ceilf(cand * s1) + 4;
            ext[A2] = sp2 + (int)ceilf(cand * s2) + 4;
            const int vol = (ext[0] + 2 * CV) * ext[1] * ext[2];
            if (vol <= cap) {
                S = cand;
                break;
            }
        }
        if (S == 0) return false;
    }
    const int Z0 = sgn > 0 ? sh.red[0] : sh.red[1] + 1;
    const int K = !any_ray ? 0 : (sgn > 0 ? (sh.red[3] - Z0) / S + 1 : (Z0 - 1 - sh.red[2]) / S + 1);
    int k_last = 0;
    if (act) k_last = min(max(sgn > 0 ? (zl - Z0) / S : (Z0 - 1 - zl) / S, 0), K - 1);

    // ---- per-ray state --------------------------------------------------------------
    const float om = act ? ff_to_f(ray.o[M]) : 0.0f;
    const float inv_dm = act ? 1.0f / ray.d[M].hi : 0.0f;
    const float tinf = act ? ff_to_f(ray.tin) : 0.0f;
    const float inv_step = 1.0f / ff_to_f(R.step);
    Accum acc = {0.0f, 0.0f, 0.0f, 1.0f, -VR_INF};
    unsigned nexec = 0, nskip = 0;
    bool stopped = false;
    // sample ranges: slab it holds [ks, ke0); slab it+1 [ke0, ke1); slab it+2 [ke1, ke2)
    int ks = 0, ke0 = 0, ke1 = 0;
    auto slab_end = [&](int k, int kprev) -> int {
        if (!act || stopped) return kprev;
        if (k >= k_last) return ray.n;
        const SlabGeo<M> g = slab_geo<M>(k, Z0, S, sgn, rf, cf);
        const float kf = ceilf(((g.zexit - om) * inv_dm - tinf) * inv_step - 0.5f);
        return kf < (float)kprev ? kprev : (kf > (float)ray.n ? ray.n : (int)kf);
    };
    // bounds of slab k for samples [k0, k1): reduce into descriptor k % VR_RING
    auto slab_bounds = [&](int k, int k0, int k1) {
        int mn[3] = {VR_BIG, VR_BIG, VR_BIG}, mx[3] = {-VR_BIG, -VR_BIG, -VR_BIG};
        if (k1 > k0) {
            const SlabGeo<M> g = slab_geo<M>(k, Z0, S, sgn, rf, cf);
            float A[3], lo[3], hi[3], w[3];
            slab_anchor(R, ray, k0, g.B0, A, lo, hi);
            const int jl = k1 - 1 - k0;
            const float jfl = (float)jl + ((k1 == ray.n && jl > 0) ? ray.last_adj : 0.0f);
            const float p1[3] = {__builtin_fmaf(jfl, ray.dd[0], A[0]),
                                 __builtin_fmaf(jfl, ray.dd[1], A[1]),
                                 __builtin_fmaf(jfl, ray.dd[2], A[2])};
            int i0[3], i1[3];
            floor_idx<INTERP>(A, lo, hi, i0, w);
            floor_idx<INTERP>(p1, lo, hi, i1, w);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(i0[a], i1[a]);
                mx[a] = max(i0[a], i1[a]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = wave_min(mn[a]);
            mx[a] = wave_max(mx[a]);
        }
        if (lane == 0 && mn[0] != VR_BIG) {
            SlabDesc& d = sh.d[k % VR_RING];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                atomicMin(&d.bmin[a], mn[a]);
                atomicMax(&d.bmax[a], mx[a]);
            }
        }
    };
    // skip-grid words of slab k's cells: issue the loads (one cell row per thread)
    const int Cx = 4 * R.cube.bx, Cy = 4 * R.cube.by;
    auto bits_issue = [&](int k, uint32_t& w0, uint32_t& w1, uint32_t& mask0, uint32_t& mask1,
                          bool& wide) {
        w0 = w1 = mask0 = mask1 = 0u;
        wide = false;
        const SlabGeo<M> g = slab_geo<M>(k, Z0, S, sgn, rf, cf);
        const SlabDesc& d = sh.d[k % VR_RING];
        if (d.bmin[0] > d.bmax[0]) return;
        int c0[3], c1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c0[a] = min(max(g.B0[a] + d.bmin[a], 0), N[a] - 1) >> 3;
            c1[a] = min(max(g.B0[a] + d.bmax[a], 0), N[a] - 1) >> 3;
        }
        const int ny_ = c1[1] - c0[1] + 1, nrow = ny_ * (c1[2] - c0[2] + 1);
        if (tid >= nrow) return;
        const int cy = c0[1] + tid % ny_, cz = c0[2] + tid / ny_;
        const int64_t b0 = ((int64_t)cz * Cy + cy) * Cx + c0[0];
        const int64_t b1 = b0 + (c1[0] - c0[0]);
        const int64_t wa = b0 >> 5, wb = b1 >> 5;
        if (wb - wa > 1) {
            wide = true;  // more than two words: treated as active
            return;
        }
        const uint32_t lo_bit = (uint32_t)(b0 & 31), hi_bit = (uint32_t)(b1 & 31);
        if (wa == wb) {
            mask0 = (hi_bit == 31 ? 0xffffffffu : ((1u << (hi_bit + 1)) - 1u)) & ~((1u << lo_bit) - 1u);
        } else {
            mask0 = ~((1u << lo_bit) - 1u);
            mask1 = hi_bit == 31 ? 0xffffffffu : ((1u << (hi_bit + 1)) - 1u);
            w1 = R.cube.cellbits[wb];
        }
        w0 = R.cube.cellbits[wa];
    };
    // box DMA of slab k into buffer k & 1
    auto box_dma = [&](int k) {
        const SlabGeo<M> g = slab_geo<M>(k, Z0, S, sgn, rf, cf);
        const SlabDesc& d = sh.d[k % VR_RING];
        const BoxGeo b = box_geo<DT, INTERP>(d, g.B0);
        if (b.empty || !d.any || b.elems > cap) return;
        uint8_t* buf = boxes + (k & 1) * R.box_bytes;
        const int total = b.nc * b.bdim[1] * b.bdim[2];
        const float inv_nc = 1.0f / (float)b.nc, inv_b1 = 1.0f / (float)b.bdim[1];
        for (int q0 = wave * 64; q0 < total; q0 += VR_WG) {
            const int q = q0 + lane;
            if (q < total) {
                const int rowi = div_small(q, b.nc, inv_nc);
                const int c = q - rowi * b.nc;
                const int iz = div_small(rowi, b.bdim[1], inv_b1);
                const int iy = rowi - iz * b.bdim[1];
                const int gy = min(b.g0[1] + iy, N[1] - 1), gz = min(b.g0[2] + iz, N[2] - 1);
                const int x = b.xa + c * CV;
                const int bxb = min(x >> 5, R.cube.bx - 1);
                const int lx = x - 32 * bxb;
                const uint64_t slot = ((uint64_t)(gz >> 5) * R.cube.by + (gy >> 5)) * R.cube.bx + bxb;
                const uint8_t* src = R.cube.pool + slot * R.cube.stride +
                                     (uint64_t)(((gz & 31) * VR_BRICK_APRON + (gy & 31)) * R.cube.row + lx) * ELEM;
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (__attribute__((address_space(3))) void*)(buf + q0 * 16),
                                                 16, 0, 0);
            }
        }
    };

    // ---- prologue: slabs 0 and 1 ------------------------------------------------------
    if (K > 0) {
        ke0 = slab_end(0, 0);
        slab_bounds(0, 0, ke0);
        if (K > 1) {
            ke1 = slab_end(1, ke0);
            slab_bounds(1, ke0, ke1);
        }
    }
    __syncthreads();
    if (R.use_skip) {
        for (int k = 0; k < min(K, 2); ++k) {
            uint32_t w0, w1, m0, m1;
            bool wide;
            bits_issue(k, w0, w1, m0, m1, wide);
            if (wide || (w0 & m0) || (w1 & m1)) sh.d[k % VR_RING].any = 1;
        }
        __syncthreads();
    }
    if (K > 0) box_dma(0);

    // ---- slab pipeline -----------------------------------------------------------------
    for (int it = 0; it < K; ++it) {
        int ke2 = ke1;
        if (it + 2 < K) {
            ke2 = slab_end(it + 2, ke1);
            slab_bounds(it + 2, ke1, ke2);
        }
        if (tid == 0) {
            if (it + 3 < K) {
                SlabDesc& d = sh.d[(it + 3) % VR_RING];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    d.bmin[a] = VR_BIG;
                    d.bmax[a] = -VR_BIG;
                }
                d.any = R.use_skip ? 0 : 1;
            }
            sh.alive[it % 3] = 0;
        }
        __builtin_amdgcn_s_waitcnt(0);  // own box copies of slab it have landed
        __syncthreads();
        if (it > 0 && sh.alive[(it - 1) % 3] == 0) break;
        uint32_t bw0 = 0, bw1 = 0, bm0 = 0, bm1 = 0;
        bool bwide = false;
        if (R.use_skip && it + 2 < K) bits_issue(it + 2, bw0, bw1, bm0, bm1, bwide);
        if (it + 1 < K) box_dma(it + 1);
        // ---- sample slab it
        {
            const SlabGeo<M> g = slab_geo<M>(it, Z0, S, sgn, rf, cf);
            const SlabDesc& d = sh.d[it % VR_RING];
            const BoxGeo b = box_geo<DT, INTERP>(d, g.B0);
            const int cnt_s = ke0 - ks;
            if (cnt_s > 0 && !stopped) {
                if (!d.any) {
                    nskip += (unsigned)cnt_s;
                } else {
                    const bool staged = b.elems <= cap;
                    const VT* box = (const VT*)(boxes + (it & 1) * R.box_bytes);
                    const int sy = b.pitch, sz = b.pitch * b.bdim[1];
                    const int xoff = g.B0[0] - b.xa;
                    float A[3], lo[3], hi[3];
                    slab_anchor(R, ray, ks, g.B0, A, lo, hi);
                    for (int j = 0; j < cnt_s; ++j) {
                        const bool last = (ks + j == ray.n - 1);
                        const float jf = (float)j + ((last && j > 0) ? ray.last_adj : 0.0f);
                        const float p[3] = {__builtin_fmaf(jf, ray.dd[0], A[0]),
                                            __builtin_fmaf(jf, ray.dd[1], A[1]),
                                            __builtin_fmaf(jf, ray.dd[2], A[2])};
                        int i[3];
                        float w[3];
                        floor_idx<INTERP>(p, lo, hi, i, w);
                        float v;
                        if (staged) {
                            const int idx = ((i[2] - b.blo[2]) * b.bdim[1] + (i[1] - b.blo[1])) * b.pitch +
                                            (i[0] + xoff);
                            v = interp_at<DT, INTERP>(box + idx, sy, sz, w[0], w[1], w[2]);
                        } else {
                            v = interp_at<DT, INTERP>(
                                pool_ptr<DT>(R.cube, g.B0[0] + i[0], g.B0[1] + i[1], g.B0[2] + i[2]),
                                R.cube.row, VR_BRICK_APRON * R.cube.row, w[0], w[1], w[2]);
                        }
                        ++nexec;
                        if (MODE == 1) {
                            acc.m = fmaxf(acc.m, v);
                        } else if (composite(R, tfl, v, last, ray, acc)) {
                            stopped = true;
                            break;
                        }
                    }
                }
            }
        }
        if (R.use_skip && it + 2 < K && (bwide || (bw0 & bm0) || (bw1 & bm1)))
            sh.d[(it + 2) % VR_RING].any = 1;
        const bool done = !act || stopped || ke0 >= ray.n;
        if (__ballot(!done) != 0ull && lane == 0) sh.alive[it % 3] = 1;
        ks = ke0;
        ke0 = ke1;
        ke1 = ke2;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (inimg) store_pixel<MODE>(R, px, py, act, acc);
    if (act) {
        cnt.nominal += (unsigned)ray.n;
        cnt.exec += nexec;
        cnt.hit += 1u;
        cnt.ert += stopped ? 1u : 0u;
        cnt.skipped += nskip;
    }
    return true;
}

// Returns false (having rendered nothing) when the tile's rays do not share a
// direction along one axis, or no slab box fits; the caller then runs the
// per-ray walker.
template <int MODE, int DT, int INTERP>
__device__ __forceinline__ bool render_tile(const DevReq& R, const int tx, const int ty,
                                            const float* __restrict__ tfl,
                                            uint8_t* __restrict__ boxes, TileShared& sh,
                                            LaneCounts& cnt) {
    const int tid = threadIdx.x;
    int px, py;
    tile_pixel(R, tx, ty, px, py);
    const bool inimg = px < R.W && py < R.H;
    if (tid == 0) {
        sh.red[0] = VR_BIG;
        sh.red[1] = -VR_BIG;
        sh.red[2] = VR_BIG;
        sh.red[3] = -VR_BIG;
        sh.red[4] = VR_BIG;
        sh.red[5] = -VR_BIG;
        sh.red[6] = VR_BIG;
        sh.red[7] = -VR_BIG;
        sh.red[8] = 0;
        sh.red[9] = 0;
        sh.red[10] = 1;
        for (int q = 0; q < VR_RING; ++q) {
            for (int a = 0; a < 3; ++a) {
                sh.d[q].bmin[a] = VR_BIG;
                sh.d[q].bmax[a] = -VR_BIG;
            }
            sh.d[q].any = R.use_skip ? 0 : 1;
        }
        sh.alive[0] = sh.alive[1] = sh.alive[2] = 0;
    }
    Ray ray;
    ray.n = 0;
    if (inimg) ray_setup(R, px, py, ray);
    // tile reference ray (identical in every lane) fixes the major axis and slab origins
    ff oc[3], dc[3];
    ray_dir(R.cam, (float)(tx * VR_TW) + 0.5f * VR_TW, (float)(ty * VR_TH) + 0.5f * VR_TH, oc, dc);
    const float ad0 = fabsf(dc[0].hi), ad1 = fabsf(dc[1].hi), ad2 = fabsf(dc[2].hi);
    const int m = (ad2 > ad0 && ad2 > ad1) ? 2 : (ad1 > ad0 ? 1 : 0);
    const float dm = m == 0 ? dc[0].hi : (m == 1 ? dc[1].hi : dc[2].hi);
    const int sgn = dm > 0.0f ? 1 : -1;
    __syncthreads();
    if (m == 0)
        return tile_march<MODE, DT, INTERP, 0>(R, ray, px, py, inimg, oc, dc, sgn, tfl, boxes, sh, cnt);
    if (m == 1)
        return tile_march<MODE, DT, INTERP, 1>(R, ray, px, py, inimg, oc, dc, sgn, tfl, boxes, sh, cnt);
    return tile_march<MODE, DT, INTERP, 2>(R, ray, px, py, inimg, oc, dc, sgn, tfl, boxes, sh, cnt);
}

// One tile: slab-staged if possible, else one independent walker per ray.
template <int MODE, int DT, int INTERP>
__device__ __forceinline__ void render_tile_any(const DevReq& R, const int tx, const int ty,
                                                const float* __restrict__ tfl,
                                                uint8_t* __restrict__ boxes, TileShared& sh,
                                                LaneCounts& cnt) {
    if (render_tile<MODE, DT, INTERP>(R, tx, ty, tfl, boxes, sh, cnt)) return;
    int px, py;
    tile_pixel(R, tx, ty, px, py);
    if (px < R.W && py < R.H) render_lane_direct<MODE, DT, INTERP>(R, px, py, tfl, cnt);
}

__device__ __forceinline__ void flush_counts(const LaneCounts& c, DevCounters* cnt,
                                             unsigned* wg /* 5 LDS words */) {
    atomicAdd(&wg[0], c.nominal);
    atomicAdd(&wg[1], c.exec);
    atomicAdd(&wg[2], c.hit);
    atomicAdd(&wg[3], c.ert);
    atomicAdd(&wg[4], c.skipped);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&cnt->samples_nominal, (unsigned long long)wg[0]);
        atomicAdd(&cnt->samples_exec, (unsigned long long)wg[1]);
        atomicAdd(&cnt->rays_hit, (unsigned long long)wg[2]);
        atomicAdd(&cnt->rays_ert, (unsigned long long)wg[3]);
        atomicAdd(&cnt->cells_skipped, (unsigned long long)wg[4]);
    }
}

// dynamic LDS: transfer-function rows (n x 32 bytes), then two slab boxes
template <int MODE, int DT, int INTERP>
__global__ __launch_bounds__(VR_WG) void k_render(const DevReq R, DevCounters* cnt) {
    extern __shared__ float4 lds4[];
    __shared__ unsigned wgc[5];
    __shared__ TileShared sh;
    float* tfl = (float*)lds4;
    const int tf_bytes = MODE == 0 ? 32 * R.tf.n : 0;
    if (MODE == 0) {
        const float4* rows = (const float4*)R.tf.rows;
        for (int e = threadIdx.x; e < 2 * R.tf.n; e += VR_WG) lds4[e] = rows[e];
    }
    if (cnt && threadIdx.x < 5) wgc[threadIdx.x] = 0u;
    __syncthreads();
    const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
    const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
    LaneCounts c = {0u, 0u, 0u, 0u, 0u};
    render_tile_any<MODE, DT, INTERP>(R, tx, ty, tfl, (uint8_t*)lds4 + tf_bytes, sh, c);
    if (cnt) flush_counts(c, cnt, wgc);
}

__global__ void k_reset_head(unsigned* head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *head = 0u;
}

template <int MODE, int DT>
__device__ __forceinline__ void dispatch_interp(const DevReq& R, int tx, int ty, float* tfl,
                                                TileShared& sh, LaneCounts& c) {
    uint8_t* boxes = (uint8_t*)tfl + (MODE == 0 ? 32 * R.tf.n : 0);
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
__global__ __launch_bounds__(VR_WG) void k_render_batch(const DevReq* __restrict__ reqs,
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
        if (R.mode == 0) {
            const float4* rows = (const float4*)R.tf.rows;
            for (int e = threadIdx.x; e < 2 * R.tf.n; e += VR_WG) lds4[e] = rows[e];
        }
        __syncthreads();
        const int tx = item.tile % R.tiles_x, ty = item.tile / R.tiles_x;
        LaneCounts c = {0u, 0u, 0u, 0u, 0u};
        if (R.mode == 0) dispatch_dtype<0>(R, tx, ty, tfl, sh, c);
        else dispatch_dtype<1>(R, tx, ty, tfl, sh, c);
        if (cnt) flush_counts(c, cnt + item.req, wgc);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <int SRC, int DST>
static hipError_t launch_bb(const void* src, int64_t nx, int64_t ny, int64_t nz, int64_t z_first,
                            int bz, int Bx, int By, uint8_t* pool, uint64_t stride, int row,
                            float* cell_minmax, float sigma, hipStream_t s) {
    hipLaunchKernelGGL((k_brick_build<SRC, DST>), dim3(Bx * By), dim3(VR_BB_WG), 0, s, src, nx,
                       ny, nz, z_first, bz, Bx, By, pool, stride, row, cell_minmax, sigma);
    return hipGetLastError();
}

hipError_t vr_launch_brick_build(int src_kind, int dst, const void* src, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t z_first, int bz, int Bx, int By,
                                 uint8_t* pool, uint64_t stride, int row, float* cell_minmax,
                                 float sigma, hipStream_t s) {
#define VR_BB(S, D)                                                                          \
    if (src_kind == S && dst == D)                                                           \
        return launch_bb<S, D>(src, nx, ny, nz, z_first, bz, Bx, By, pool, stride, row,      \
                               cell_minmax, sigma, s);
    VR_BB(0, 0)
    VR_BB(0, 1)
    VR_BB(0, 2)
    VR_BB(1, 1)
    VR_BB(2, 2)
#undef VR_BB
    return hipErrorInvalidValue;
}

hipError_t vr_launch_classify(const float* cell_minmax, uint64_t* mask, uint32_t* cellbits,
                              int Bx, int By, int Bz, int mode, float clip, float scale,
                              float bias, int n, const int* kpos, hipStream_t s) {
    const int nslots = Bx * By * Bz;
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3((nslots + VR_BB_WG - 1) / VR_BB_WG), dim3(VR_BB_WG), 0, s,
                       cell_minmax, mask, nslots, mode, clip, scale, bias, n, kpos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nwords = vr_cellbits_words(Bx, By, Bz);
    hipLaunchKernelGGL(k_cellbits, dim3((nwords + VR_BB_WG - 1) / VR_BB_WG), dim3(VR_BB_WG), 0, s,
                       (const uint64_t*)mask, cellbits, nwords, Bx, By);
    return hipGetLastError();
}

template <int MODE, int DT, int INTERP>
static hipError_t launch_r(const DevReq& R, DevCounters* cnt, hipStream_t s) {
    const int grid = R.tiles_x * R.tiles_y;
    const size_t lds = (MODE == 0 ? (size_t)R.tf.n * 32 : 0) + 2 * (size_t)R.box_bytes;
    hipLaunchKernelGGL((k_render<MODE, DT, INTERP>), dim3(grid), dim3(VR_WG), lds, s, R, cnt);
    return hipGetLastError();
}

hipError_t vr_launch_render(const DevReq& R, DevCounters* cnt, hipStream_t s) {
    const int key = R.mode * 100 + R.cube.dtype * 10 + R.interp;
    switch (key) {
        case 0: return launch_r<0, 0, 0>(R, cnt, s);
        case 1: return launch_r<0, 0, 1>(R, cnt, s);
        case 10: return launch_r<0, 1, 0>(R, cnt, s);
        case 11: return launch_r<0, 1, 1>(R, cnt, s);
        case 20: return launch_r<0, 2, 0>(R, cnt, s);
        case 21: return launch_r<0, 2, 1>(R, cnt, s);
        case 100: return launch_r<1, 0, 0>(R, cnt, s);
        case 101: return launch_r<1, 0, 1>(R, cnt, s);
        case 110: return launch_r<1, 1, 0>(R, cnt, s);
        case 111: return launch_r<1, 1, 1>(R, cnt, s);
        case 120: return launch_r<1, 2, 0>(R, cnt, s);
        case 121: return launch_r<1, 2, 1>(R, cnt, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t vr_launch_batch(const DevReq* reqs, const DevItem* items, const int* nitems,
                           unsigned* head, DevCounters* cnt, size_t lds_bytes, int grid,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, head);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_render_batch, dim3(grid), dim3(VR_WG), lds_bytes, s, reqs, items, nitems,
                       head, cnt);
    return hipGetLastError();
}
