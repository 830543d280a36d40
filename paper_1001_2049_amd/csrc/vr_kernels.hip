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

// Launch-shape tuning (compile-time): extra dynamic LDS per workgroup (caps
// workgroups per CU), tile order, and paired x-neighbour loads.
#ifndef VR_EXTRA_LDS
#define VR_EXTRA_LDS 0
#endif
#ifndef VR_TILE_MAP
#define VR_TILE_MAP 0
#endif
#ifndef VR_PAIR_LOADS
#define VR_PAIR_LOADS 0
#endif
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

// src_kind: 0 float32 values, 1 f16 codes, 2 bf16 codes (copied as-is)
template <int SRC, int DST>
__global__ __launch_bounds__(VR_WG) void k_brick_build(
    const void* __restrict__ src, int64_t nx, int64_t ny, int64_t nz, int64_t z_first, int bz,
    int Bx, int By, const uint32_t* __restrict__ slot_of_brick, uint8_t* __restrict__ pool,
    uint64_t stride, float* __restrict__ cell_minmax, float sigma) {
    __shared__ float vals[VR_BRICK_VOX];
    __shared__ float cmin[VR_CELLS_PER_BRICK], cmax[VR_CELLS_PER_BRICK];
    const int bxi = blockIdx.x % Bx, byi = blockIdx.x / Bx;
    const uint32_t slot = slot_of_brick[((int64_t)bz * By + byi) * Bx + bxi];
    typedef typename Vox<DST>::T DT;
    DT* dst = (DT*)(pool + (uint64_t)slot * stride);
    const int64_t x0 = (int64_t)bxi * VR_BRICK, y0 = (int64_t)byi * VR_BRICK,
                  z0 = (int64_t)bz * VR_BRICK;
    for (int e = threadIdx.x; e < VR_BRICK_VOX; e += VR_WG) {
        const int lx = e % VR_BRICK_APRON, ly = (e / VR_BRICK_APRON) % VR_BRICK_APRON,
                  lz = e / (VR_BRICK_APRON * VR_BRICK_APRON);
        int64_t gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        gx = gx < nx - 1 ? gx : nx - 1;
        gy = gy < ny - 1 ? gy : ny - 1;
        gz = gz < nz - 1 ? gz : nz - 1;
        const int64_t si = ((gz - z_first) * ny + gy) * nx + gx;
        float dec;
        if (SRC == 0) {
            float v = ((const float*)src)[si];
            if (DST == 0) {
                float s = v / sigma;
                ((float*)dst)[e] = s;
                dec = s;
            } else if (DST == 1) {
                uint16_t c = enc_f16(v / sigma);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<1>::dec(c);
            } else {
                uint16_t c = enc_bf16(v / sigma);
                ((uint16_t*)dst)[e] = c;
                dec = Vox<2>::dec(c);
            }
        } else {
            uint16_t c = ((const uint16_t*)src)[si];
            ((uint16_t*)dst)[e] = c;
            dec = Vox<DST>::dec(c);
        }
        vals[e] = dec;
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
        float* cm = cell_minmax + (uint64_t)slot * (2 * VR_CELLS_PER_BRICK);
        cm[2 * threadIdx.x] = cmin[threadIdx.x];
        cm[2 * threadIdx.x + 1] = cmax[threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// Skip classification: one thread per slot
// ---------------------------------------------------------------------------
// EA: a cell may contribute iff some value v in [max(min, clip), max] maps to a
// table interval with a non-zero kappa at either end.  The value->u map is
// evaluated with exactly the float operations the render kernel uses, so the
// test is conservative for every sample the kernel can produce.
// MIP: a cell may raise the projected maximum above the clip iff max >= clip.
__global__ __launch_bounds__(VR_WG) void k_classify(const float* __restrict__ cell_minmax,
                                                    uint64_t* __restrict__ mask, int nslots,
                                                    int mode, float clip, float scale,
                                                    float bias, int n,
                                                    const int* __restrict__ kpos) {
    const int s = blockIdx.x * VR_WG + threadIdx.x;
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

// ---------------------------------------------------------------------------
// Rendering
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

template <int MODE, int DT, int INTERP>
__device__ __forceinline__ void render_lane(const DevReq& R, const int px, const int py,
                                            const float* __restrict__ tfl, LaneCounts& cnt) {
    typedef typename Vox<DT>::T VT;
    const DevCam& cam = R.cam;
    const float fi = (float)px + 0.5f, fj = (float)py + 0.5f;
    ff o[3], d[3];
    if (cam.ortho) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = ff_add(ff_add(cam.o[a], ff_mul_f(cam.dx[a], fi)), ff_mul_f(cam.dy[a], fj));
            d[a] = cam.dir[a];
        }
    } else {
        ff dir[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            dir[a] = ff_add(ff_add(cam.base[a], ff_mul_f(cam.dx[a], fi)), ff_mul_f(cam.dy[a], fj));
        const ff n2 = ff_add(ff_add(ff_mul(dir[0], dir[0]), ff_mul(dir[1], dir[1])),
                             ff_mul(dir[2], dir[2]));
        const ff inv = ff_div(ff_make(1.0f), ff_sqrt(n2));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d[a] = ff_mul(dir[a], inv);
            o[a] = cam.o[a];
        }
    }
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    const int B[3] = {R.cube.bx, R.cube.by, R.cube.bz};
    ff tin = cam.ortho ? ff_make(-VR_INF) : ff_make(0.0f);
    ff tout = ff_make(VR_INF);
    bool hit = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hib = (float)N[a] - 0.5f;
        if (d[a].hi != 0.0f) {
            const ff t0 = ff_div(ff_sub(ff_make(-0.5f), o[a]), d[a]);
            const ff t1 = ff_div(ff_sub(ff_make(hib), o[a]), d[a]);
            tin = ff_max(tin, ff_min(t0, t1));
            tout = ff_min(tout, ff_max(t0, t1));
        } else if (ff_lt(o[a], ff_make(-0.5f)) || ff_lt(ff_make(hib), o[a])) {
            hit = false;
        }
    }
    hit = hit && ff_lt(tin, tout);
    float* out = R.out;
    const int64_t pix = (int64_t)py * R.W + px;
    if (!hit) {
        if (MODE == 0) {
            *(float4*)(out + 4 * pix) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            out[pix] = -VR_INF;
        }
        return;
    }
    // lattice: n segments of length step, the last one shortened
    const ff L = ff_sub(tout, tin);
    const ff rr = ff_div(L, R.step);
    float nf = ceilf(rr.hi);
    if (nf == rr.hi && rr.lo > 0.0f) nf += 1.0f;
    const int n = nf < 1.0f ? 1 : (int)nf;
    const float stepf = ff_to_f(R.step);
    float len_last = ff_to_f(ff_sub(L, ff_mul_f(R.step, (float)(n - 1))));
    len_last = fmaxf(len_last, 0.0f);
    // the last segment's midpoint sits last_adj lattice steps before a full step's
    const float last_adj = 0.5f * (len_last / stepf - 1.0f);
    const float c_full = -stepf * VR_LOG2E, c_last = -len_last * VR_LOG2E;
    float dd[3], inv_dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dd[a] = ff_to_f(ff_mul(d[a], R.step));
        inv_dd[a] = dd[a] != 0.0f ? 1.0f / dd[a] : 0.0f;
    }
    const float shift = INTERP == 0 ? 0.5f : 0.0f;  // nearest: cells bounded at 8c - 1/2

    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f, mval = -VR_INF;
    int k0 = 0, m = 0, j = 0;
    float A[3] = {0.0f, 0.0f, 0.0f}, hb[3] = {0.0f, 0.0f, 0.0f};
    const uint8_t* base = nullptr;
    uint64_t mask = 0;
    unsigned nexec = 0, nskip = 0;
    bool stopped = false;
    const float tf_scale = R.tf.scale, tf_bias = R.tf.bias, clip = R.tf.clip;
    const float tf_nm1 = (float)(R.tf.n - 1), tf_nm2 = (float)(R.tf.n - 2);

    while (true) {
        if (j >= m) {
            // enter the brick holding sample k0; anchor local coordinates there
            k0 += m;
            if (k0 >= n) break;
            ff t = ff_add(tin, ff_mul_f(R.step, (float)k0 + 0.5f));
            if (k0 == n - 1) t = ff_add(t, ff_make(last_adj * stepf));
            int b[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const ff P = ff_add(o[a], ff_mul(t, d[a]));
                int bb = (int)floorf(P.hi * (1.0f / VR_BRICK));
                bb = bb < 0 ? 0 : (bb > B[a] - 1 ? B[a] - 1 : bb);
                b[a] = bb;
                A[a] = ff_to_f(ff_add(P, ff_make(-(float)(VR_BRICK * bb))));
                hb[a] = fminf(31.999998f, (float)(N[a] - 1 - VR_BRICK * bb));
            }
            float s = VR_INF;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (dd[a] > 0.0f && b[a] < B[a] - 1) s = fminf(s, ((float)VR_BRICK - A[a]) * inv_dd[a]);
                if (dd[a] < 0.0f && b[a] > 0) s = fminf(s, (-A[a]) * inv_dd[a]);
            }
            const int rem = n - k0;
            m = s >= (float)rem ? rem : max(1, (int)ceilf(s));
            j = 0;
            const uint32_t slot =
                R.cube.slot_of_brick[((int64_t)b[2] * B[1] + b[1]) * B[0] + b[0]];
            base = R.cube.pool + (uint64_t)slot * R.cube.stride;
            mask = R.use_skip ? R.cube.mask[slot] : ~0ull;
            if (mask == 0) {
                nskip += m;
                j = m;
                continue;
            }
        }
        const bool last = (k0 + j == n - 1);
        const float jf = (float)j + ((last && j > 0) ? last_adj : 0.0f);
        const float p0 = __builtin_fmaf(jf, dd[0], A[0]);
        const float p1 = __builtin_fmaf(jf, dd[1], A[1]);
        const float p2 = __builtin_fmaf(jf, dd[2], A[2]);
        const float q0 = __builtin_amdgcn_fmed3f(p0, 0.0f, hb[0]);
        const float q1 = __builtin_amdgcn_fmed3f(p1, 0.0f, hb[1]);
        const float q2 = __builtin_amdgcn_fmed3f(p2, 0.0f, hb[2]);
        int i0, i1, i2;
        float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
        int cell;
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
                if (dd[a] > 0.0f)
                    s = fminf(s, ((float)(VR_CELL * (c3[a] + 1)) - 1e-4f - pw[a]) * inv_dd[a]);
                else if (dd[a] < 0.0f)
                    s = fminf(s, ((float)(VR_CELL * c3[a]) + 1e-4f - pw[a]) * inv_dd[a]);
            }
            const int jump = s >= 1.0e6f ? (1 << 20) : max(1, (int)ceilf(s));
            nskip += min(jump, m - j);
            j += jump;
            continue;
        }
        const int idx = (i2 * VR_BRICK_APRON + i1) * VR_BRICK_APRON + i0;
        const VT* __restrict__ bp = (const VT*)base + idx;
        float v;
        if (INTERP == 1 && DT == 0 && VR_PAIR_LOADS) {
            typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
            const float* fp = (const float*)bp;
            const f2u a00 = *(const f2u*)(fp);
            const f2u a10 = *(const f2u*)(fp + VR_BRICK_APRON);
            const f2u a01 = *(const f2u*)(fp + VR_BRICK_APRON * VR_BRICK_APRON);
            const f2u a11 = *(const f2u*)(fp + VR_BRICK_APRON * VR_BRICK_APRON + VR_BRICK_APRON);
            const float x00 = __builtin_fmaf(w0, a00.y - a00.x, a00.x);
            const float x10 = __builtin_fmaf(w0, a10.y - a10.x, a10.x);
            const float x01 = __builtin_fmaf(w0, a01.y - a01.x, a01.x);
            const float x11 = __builtin_fmaf(w0, a11.y - a11.x, a11.x);
            const float y0 = __builtin_fmaf(w1, x10 - x00, x00);
            const float y1 = __builtin_fmaf(w1, x11 - x01, x01);
            v = __builtin_fmaf(w2, y1 - y0, y0);
        } else if (INTERP == 1) {
            const float c000 = Vox<DT>::dec(bp[0]);
            const float c100 = Vox<DT>::dec(bp[1]);
            const float c010 = Vox<DT>::dec(bp[VR_BRICK_APRON]);
            const float c110 = Vox<DT>::dec(bp[VR_BRICK_APRON + 1]);
            const float c001 = Vox<DT>::dec(bp[VR_BRICK_APRON * VR_BRICK_APRON]);
            const float c101 = Vox<DT>::dec(bp[VR_BRICK_APRON * VR_BRICK_APRON + 1]);
            const float c011 = Vox<DT>::dec(bp[VR_BRICK_APRON * VR_BRICK_APRON + VR_BRICK_APRON]);
            const float c111 =
                Vox<DT>::dec(bp[VR_BRICK_APRON * VR_BRICK_APRON + VR_BRICK_APRON + 1]);
            const float x00 = __builtin_fmaf(w0, c100 - c000, c000);
            const float x10 = __builtin_fmaf(w0, c110 - c010, c010);
            const float x01 = __builtin_fmaf(w0, c101 - c001, c001);
            const float x11 = __builtin_fmaf(w0, c111 - c011, c011);
            const float y0 = __builtin_fmaf(w1, x10 - x00, x00);
            const float y1 = __builtin_fmaf(w1, x11 - x01, x01);
            v = __builtin_fmaf(w2, y1 - y0, y0);
        } else {
            v = Vox<DT>::dec(bp[0]);
        }
        ++nexec;
        ++j;
        if (MODE == 1) {
            mval = fmaxf(mval, v);
            continue;
        }
        // classify: clamp-interpolated table row; values below the clip are empty
        float u = __builtin_fmaf(v, tf_scale, tf_bias);
        u = __builtin_amdgcn_fmed3f(u, 0.0f, tf_nm1);
        const float fl = fminf(floorf(u), tf_nm2);
        const float g = u - fl;
        const float4* row = (const float4*)(tfl + 8 * (int)fl);
        const float4 r0 = row[0], dr = row[1];
        float kap = __builtin_fmaf(g, dr.w, r0.w);
        kap = v < clip ? 0.0f : kap;
        // emission-absorption over the segment: alpha = 1 - exp(-kappa len)
        const float ex = __builtin_amdgcn_exp2f(kap * (last ? c_last : c_full));
        const float wgt = T * (1.0f - ex);
        C0 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.x, r0.x), C0);
        C1 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.y, r0.y), C1);
        C2 = __builtin_fmaf(wgt, __builtin_fmaf(g, dr.z, r0.z), C2);
        T *= ex;
        if (T <= R.ert_T) {
            stopped = true;
            break;
        }
    }
    if (MODE == 0) {
        *(float4*)(out + 4 * pix) = make_float4(C0, C1, C2, 1.0f - T);
    } else {
        out[pix] = (mval >= clip) ? mval * R.out_scale : 0.0f;
    }
    cnt.nominal += (unsigned)n;
    cnt.exec += nexec;
    cnt.hit += 1u;
    cnt.ert += stopped ? 1u : 0u;
    cnt.skipped += nskip;
}

__device__ __forceinline__ void flush_counts(const LaneCounts& c, DevCounters* cnt,
                                             unsigned* wg /* 5 LDS words */) {
    // wave-level sums first (64-bit safe: per-lane values are below 2^26)
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

template <int MODE, int DT, int INTERP>
__global__ __launch_bounds__(VR_WG) void k_render(const DevReq R, DevCounters* cnt) {
    extern __shared__ float4 tfl4[];
    __shared__ unsigned wgc[5];
    float* tfl = (float*)tfl4;
    if (MODE == 0) {
        const float4* rows = (const float4*)R.tf.rows;
        for (int e = threadIdx.x; e < 2 * R.tf.n; e += VR_WG) tfl4[e] = rows[e];
    }
    if (cnt && threadIdx.x < 5) wgc[threadIdx.x] = 0u;
    __syncthreads();
#if VR_TILE_MAP == 1
    // each XCD owns a band of rows; inside it, consecutive workgroups of one CU
    // (XCD-local ids k, k+32, ...) take a 2-tile-wide column
    int tx, ty;
    {
        const int g = blockIdx.x, x = g & 7, k = g >> 3;
        const int per = gridDim.x >> 3;
        const int c = k & 31, sidx = k >> 5;
        const int band_rows = per / R.tiles_x;
        tx = 2 * c + (sidx & 1);
        ty = x * band_rows + (sidx >> 1);
    }
#else
    const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
    const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
#endif
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = tx * VR_TILE + (wave & 1) * 8 + (lane & 7);
    const int py = ty * VR_TILE + (wave >> 1) * 8 + (lane >> 3);
    LaneCounts c = {0u, 0u, 0u, 0u, 0u};
    if (px < R.W && py < R.H) render_lane<MODE, DT, INTERP>(R, px, py, tfl, c);
    if (cnt) flush_counts(c, cnt, wgc);
}

__global__ void k_reset_head(unsigned* head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *head = 0u;
}

template <int MODE, int DT>
__device__ __forceinline__ void dispatch_interp(const DevReq& R, int px, int py, const float* tfl,
                                                LaneCounts& c) {
    if (R.interp == 1) render_lane<MODE, DT, 1>(R, px, py, tfl, c);
    else render_lane<MODE, DT, 0>(R, px, py, tfl, c);
}

template <int MODE>
__device__ __forceinline__ void dispatch_dtype(const DevReq& R, int px, int py, const float* tfl,
                                               LaneCounts& c) {
    if (R.cube.dtype == 1) dispatch_interp<MODE, 1>(R, px, py, tfl, c);
    else if (R.cube.dtype == 2) dispatch_interp<MODE, 2>(R, px, py, tfl, c);
    else dispatch_interp<MODE, 0>(R, px, py, tfl, c);
}

// Persistent grid: each workgroup pulls (request, tile) items until the list is
// exhausted.  Which workgroup renders a tile never changes the tile's pixels.
__global__ __launch_bounds__(VR_WG) void k_render_batch(const DevReq* __restrict__ reqs,
                                                        const DevItem* __restrict__ items,
                                                        int nitems, unsigned* head,
                                                        DevCounters* cnt) {
    extern __shared__ float4 tfl4[];
    __shared__ int s_item;
    __shared__ unsigned wgc[5];
    float* tfl = (float*)tfl4;
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
            for (int e = threadIdx.x; e < 2 * R.tf.n; e += VR_WG) tfl4[e] = rows[e];
        }
        __syncthreads();
        const int tx = item.tile % R.tiles_x, ty = item.tile / R.tiles_x;
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int px = tx * VR_TILE + (wave & 1) * 8 + (lane & 7);
        const int py = ty * VR_TILE + (wave >> 1) * 8 + (lane >> 3);
        LaneCounts c = {0u, 0u, 0u, 0u, 0u};
        if (px < R.W && py < R.H) {
            if (R.mode == 0) dispatch_dtype<0>(R, px, py, tfl, c);
            else dispatch_dtype<1>(R, px, py, tfl, c);
        }
        if (cnt) flush_counts(c, cnt + item.req, wgc);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <int SRC, int DST>
static hipError_t launch_bb(const void* src, int64_t nx, int64_t ny, int64_t nz, int64_t z_first,
                            int bz, int Bx, int By, const uint32_t* slot_of_brick, uint8_t* pool,
                            uint64_t stride, float* cell_minmax, float sigma, hipStream_t s) {
    hipLaunchKernelGGL((k_brick_build<SRC, DST>), dim3(Bx * By), dim3(VR_WG), 0, s, src, nx, ny,
                       nz, z_first, bz, Bx, By, slot_of_brick, pool, stride, cell_minmax, sigma);
    return hipGetLastError();
}

hipError_t vr_launch_brick_build(int src_kind, int dst, const void* src, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t z_first, int bz, int Bx, int By,
                                 const uint32_t* slot_of_brick, uint8_t* pool, uint64_t stride,
                                 float* cell_minmax, float sigma, hipStream_t s) {
#define VR_BB(S, D)                                                                              \
    if (src_kind == S && dst == D)                                                               \
        return launch_bb<S, D>(src, nx, ny, nz, z_first, bz, Bx, By, slot_of_brick, pool, stride, \
                               cell_minmax, sigma, s);
    VR_BB(0, 0)
    VR_BB(0, 1)
    VR_BB(0, 2)
    VR_BB(1, 1)
    VR_BB(2, 2)
#undef VR_BB
    return hipErrorInvalidValue;
}

hipError_t vr_launch_classify(const float* cell_minmax, uint64_t* mask, int nslots, int mode,
                              float clip, float scale, float bias, int n, const int* kpos,
                              hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3((nslots + VR_WG - 1) / VR_WG), dim3(VR_WG), 0, s,
                       cell_minmax, mask, nslots, mode, clip, scale, bias, n, kpos);
    return hipGetLastError();
}

template <int MODE, int DT, int INTERP>
static hipError_t launch_r(const DevReq& R, DevCounters* cnt, hipStream_t s) {
    const int grid = R.tiles_x * R.tiles_y;
    const size_t lds = (MODE == 0 ? (size_t)R.tf.n * 32 : 0) + VR_EXTRA_LDS;
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

hipError_t vr_launch_batch(const DevReq* reqs, const DevItem* items, int nitems, unsigned* head,
                           DevCounters* cnt, int max_tf_n, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, head);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)(max_tf_n > 0 ? max_tf_n : 0) * 32;
    hipLaunchKernelGGL(k_render_batch, dim3(grid), dim3(VR_WG), lds, s, reqs, items, nitems, head,
                       cnt);
    return hipGetLastError();
}
