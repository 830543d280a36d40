// vr_render.h — the per-tile render machinery (ray set-up, slab staging,
// sampling, classification, compositing, store) and the single-image
// kernel template.  Included by the translation units that instantiate the
// kernels (one per render mode and storage format, and the batched kernel),
// so that they compile in parallel.
#pragma once

#include "vr_common.h"
#include "vr_launch.h"

// ---------------------------------------------------------------------------
// Rendering: shared pieces
// ---------------------------------------------------------------------------
struct LaneCounts {
    unsigned nominal, exec, hit, ert, skipped;
};

// One ray: origin/direction and chord in float-float, the sample lattice.
struct Ray {
    ff o[3], d[3];
    ff tin;
    int n;                 // lattice samples; 0 when the ray misses the cube
    int kb, ke;            // samples [kb, ke) are taken (a sub-cube window; else 0, n)
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

__device__ __forceinline__ float ff_ceil(const ff& x) {
    float c = ceilf(x.hi);
    if (c == x.hi && x.lo > 0.0f) c += 1.0f;
    return c;
}
__device__ __forceinline__ float ff_floor(const ff& x) {
    float f = floorf(x.hi);
    if (f == x.hi && x.lo < 0.0f) f -= 1.0f;
    return f;
}

// Sub-cube window: the lattice samples whose position on the window axis lies
// in [win_lo, win_hi).  Positions E + (k + 1/2) D (E the entry point, D = step
// times the direction) are monotone in k, so the samples form a range,
// found in float-float; the last sample, moved back to its short segment's
// midpoint, is tested on its own.
__device__ __forceinline__ void window_range(const DevReq& R, Ray& ray) {
    const int a = R.win_axis;
    const ff E = ff_add(a == 0 ? ray.o[0] : (a == 1 ? ray.o[1] : ray.o[2]),
                        ff_mul(ray.tin, a == 0 ? ray.d[0] : (a == 1 ? ray.d[1] : ray.d[2])));
    const ff D = ff_mul(a == 0 ? ray.d[0] : (a == 1 ? ray.d[1] : ray.d[2]), R.step);
    const int n = ray.n;
    const bool lo_inf = R.win_lo == -VR_INF, hi_inf = R.win_hi == VR_INF;
    // position of sample k (regular lattice) relative to a window edge
    auto rel = [&](float edge) { return ff_sub(ff_div(ff_sub(ff_make(edge), E), D), ff_make(0.5f)); };
    float kb, ke;
    if (D.hi > 0.0f) {
        kb = lo_inf ? 0.0f : ff_ceil(rel(R.win_lo));
        ke = hi_inf ? (float)n : ff_ceil(rel(R.win_hi));
    } else if (D.hi < 0.0f) {
        kb = hi_inf ? 0.0f : ff_floor(rel(R.win_hi)) + 1.0f;
        ke = lo_inf ? (float)n : ff_floor(rel(R.win_lo)) + 1.0f;
    } else {
        const bool in = (lo_inf || !ff_lt(E, ff_make(R.win_lo))) && (hi_inf || ff_lt(E, ff_make(R.win_hi)));
        kb = 0.0f;
        ke = in ? (float)n : 0.0f;
    }
    // the regular lattice decides samples 0 .. n-2; the last one is tested at
    // its own position
    kb = fminf(fmaxf(kb, 0.0f), (float)(n - 1));
    ke = fminf(fmaxf(ke, 0.0f), (float)(n - 1));
    const ff pl = ff_add(E, ff_mul_f(D, (float)n - 0.5f + ray.last_adj));
    const bool last_in = (lo_inf || !ff_lt(pl, ff_make(R.win_lo))) && (hi_inf || ff_lt(pl, ff_make(R.win_hi)));
    int b = (int)kb, e = (int)ke;
    if (last_in && (e == n - 1 || b >= e)) {
        if (b >= e) b = n - 1;
        e = n;
    }
    if (b >= e) b = e = 0;
    ray.kb = b;
    ray.ke = e;
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
    ray.kb = 0;
    ray.ke = ray.n;
    if (R.win_axis >= 0) window_range(R, ray);
}

// Parameter t of lattice sample k.
__device__ __forceinline__ ff sample_t(const DevReq& R, const Ray& ray, int k) {
    ff t = ff_add(ray.tin, ff_mul_f(R.step, (float)k + 0.5f));
    if (k == ray.n - 1) t = ff_add(t, ff_make(ray.last_adj * ff_to_f(R.step)));
    return t;
}

// Element offsets of local voxel coordinates inside a slot (separable).
template <int DT>
__device__ __forceinline__ int slot_x(int lx) {
    constexpr int CV = DT == 0 ? 4 : 8;
    return (lx / CV) * 8 * CV + lx % CV;
}
template <int DT>
__device__ __forceinline__ int slot_y(int ly, int xch) {
    constexpr int CV = DT == 0 ? 4 : 8;
    return (ly >> 2) * xch * 8 * CV + (ly & 3) * CV;
}
template <int DT>
__device__ __forceinline__ int slot_z(int lz, int xch) {
    constexpr int CV = DT == 0 ? 4 : 8;
    return (lz >> 1) * VR_SLOT_YG * xch * 8 * CV + (lz & 1) * 4 * CV;
}

// Interpolated value at local voxel (lx, ly, lz) of a slot with weights w;
// the +1 neighbours are in the same slot thanks to the apron.
template <int DT, int INTERP>
__device__ __forceinline__ float slot_value(const typename Vox<DT>::T* base, int xch, int lx, int ly,
                                            int lz, float w0, float w1, float w2);

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

template <int DT, int INTERP>
__device__ __forceinline__ float slot_value(const typename Vox<DT>::T* base, int xch, int lx, int ly,
                                            int lz, float w0, float w1, float w2) {
    const int x0 = slot_x<DT>(lx), y0 = slot_y<DT>(ly, xch), z0 = slot_z<DT>(lz, xch);
    if (INTERP == 0) return Vox<DT>::dec(base[x0 + y0 + z0]);
    const int x1 = slot_x<DT>(lx + 1), y1 = slot_y<DT>(ly + 1, xch), z1 = slot_z<DT>(lz + 1, xch);
    return trilerp(Vox<DT>::dec(base[z0 + y0 + x0]), Vox<DT>::dec(base[z0 + y0 + x1]),
                   Vox<DT>::dec(base[z0 + y1 + x0]), Vox<DT>::dec(base[z0 + y1 + x1]),
                   Vox<DT>::dec(base[z1 + y0 + x0]), Vox<DT>::dec(base[z1 + y0 + x1]),
                   Vox<DT>::dec(base[z1 + y1 + x0]), Vox<DT>::dec(base[z1 + y1 + x1]), w0, w1, w2);
}

// Value of global voxel position (gx, gy, gz) (floor indices) from the pool.
template <int DT, int INTERP>
__device__ __forceinline__ float pool_value(const DevCube& c, int gx, int gy, int gz, float w0,
                                            float w1, float w2) {
    const uint32_t slot = __umul24(__umul24(gz >> 5, c.by) + (gy >> 5), c.bx) + (gx >> 5);
    const typename Vox<DT>::T* base = (const typename Vox<DT>::T*)(c.pool + (uint64_t)slot * c.stride);
    return slot_value<DT, INTERP>(base, c.xch, gx & 31, gy & 31, gz & 31, w0, w1, w2);
}

// The 8 trilinear corners at element idx of a box staged in LDS (strides 1,
// sy, sz elements), decoded to float.  16-bit storage: each pair (x, x+1) is
// cut from the two aligned dwords that hold it (row strides are multiples of
// 8 elements, so every row shares the parity of idx), keeping every LDS
// access dword-aligned.
template <int DT>
__device__ __forceinline__ void box_corners(__attribute__((address_space(3))) const typename Vox<DT>::T* box,
                                            int idx, int sy, int sz, float c[8]) {
    if (DT == 0) {
        const auto* bp = box + idx;
        c[0] = Vox<DT>::dec(bp[0]);
        c[1] = Vox<DT>::dec(bp[1]);
        c[2] = Vox<DT>::dec(bp[sy]);
        c[3] = Vox<DT>::dec(bp[sy + 1]);
        c[4] = Vox<DT>::dec(bp[sz]);
        c[5] = Vox<DT>::dec(bp[sz + 1]);
        c[6] = Vox<DT>::dec(bp[sz + sy]);
        c[7] = Vox<DT>::dec(bp[sz + sy + 1]);
        return;
    }
    typedef __attribute__((address_space(3))) const uint32_t LW;
    LW* wp = (LW*)box + (idx >> 1);
    const uint32_t sel = (idx & 1) ? 0x05040302u : 0x03020100u;
    const int hy = sy >> 1, hz = sz >> 1;
    const uint32_t p00 = __builtin_amdgcn_perm(wp[1], wp[0], sel);
    const uint32_t p10 = __builtin_amdgcn_perm(wp[hy + 1], wp[hy], sel);
    const uint32_t p01 = __builtin_amdgcn_perm(wp[hz + 1], wp[hz], sel);
    const uint32_t p11 = __builtin_amdgcn_perm(wp[hz + hy + 1], wp[hz + hy], sel);
    c[0] = Vox<DT>::dec((uint16_t)p00);
    c[1] = Vox<DT>::dec((uint16_t)(p00 >> 16));
    c[2] = Vox<DT>::dec((uint16_t)p10);
    c[3] = Vox<DT>::dec((uint16_t)(p10 >> 16));
    c[4] = Vox<DT>::dec((uint16_t)p01);
    c[5] = Vox<DT>::dec((uint16_t)(p01 >> 16));
    c[6] = Vox<DT>::dec((uint16_t)p11);
    c[7] = Vox<DT>::dec((uint16_t)(p11 >> 16));
}

// Accumulation state of one ray.
struct Accum {
    float C0, C1, C2, T, m;
};

// Classify sample value v and composite it front to back; returns true when
// the ray becomes opaque enough to stop.
__device__ __forceinline__ bool composite(const DevReq& R, const float* __restrict__ tfl, float v,
                                          bool last, const Ray& ray, Accum& acc) {
    if (v < R.tf.clip) return false;  // opacity factor 1, weight 0: no change
    float u = __builtin_fmaf(v, R.tf.scale, R.tf.bias);
    u = __builtin_amdgcn_fmed3f(u, 0.0f, (float)(R.tf.n - 1));
    // u >= 0: truncation is the floor; at u = n - 1 the last row is taken with
    // weight 0 (its difference entry is zero), which gives that row exactly
    const float g = __builtin_amdgcn_fractf(u);
    const float4* row = (const float4*)(tfl + 8 * (int)u);
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

// Two consecutive samples of one ray, composited as composite() would one
// after the other, without a branch between them: once the first makes the
// ray opaque enough to stop, the second enters with opacity factor 1 and
// weight 0, which leaves colour and transmittance exactly as they were.
// nexec counts the samples composited; returns true when the ray stops.
__device__ __forceinline__ bool composite2(const DevReq& R, const float* __restrict__ tfl, float v0,
                                           float v1, bool last1, const Ray& ray, Accum& acc,
                                           unsigned& nexec) {
    // Below the clip a sample has opacity factor exactly 1 and weight 0 and
    // changes nothing: the table rows are read only for lanes that need them.
    if (v0 < R.tf.clip && v1 < R.tf.clip) {
        nexec += 2u;
        return false;
    }
    const float hi = (float)(R.tf.n - 1);
    const float u0 = __builtin_amdgcn_fmed3f(__builtin_fmaf(v0, R.tf.scale, R.tf.bias), 0.0f, hi);
    const float u1 = __builtin_amdgcn_fmed3f(__builtin_fmaf(v1, R.tf.scale, R.tf.bias), 0.0f, hi);
    const float g0 = __builtin_amdgcn_fractf(u0), g1 = __builtin_amdgcn_fractf(u1);
    const float4* ra = (const float4*)(tfl + 8 * (int)u0);
    const float4* rb = (const float4*)(tfl + 8 * (int)u1);
    const float4 a0 = ra[0], da = ra[1], b0 = rb[0], db = rb[1];
    float k0 = __builtin_fmaf(g0, da.w, a0.w);
    float k1 = __builtin_fmaf(g1, db.w, b0.w);
    k0 = v0 < R.tf.clip ? 0.0f : k0;
    k1 = v1 < R.tf.clip ? 0.0f : k1;
    const float e0 = __builtin_amdgcn_exp2f(k0 * ray.c_full);
    const float e1r = __builtin_amdgcn_exp2f(k1 * (last1 ? ray.c_last : ray.c_full));
    const float w0 = acc.T * (1.0f - e0);
    acc.C0 = __builtin_fmaf(w0, __builtin_fmaf(g0, da.x, a0.x), acc.C0);
    acc.C1 = __builtin_fmaf(w0, __builtin_fmaf(g0, da.y, a0.y), acc.C1);
    acc.C2 = __builtin_fmaf(w0, __builtin_fmaf(g0, da.z, a0.z), acc.C2);
    const float T0 = acc.T * e0;
    const bool go = T0 > R.ert_T;
    const float e1 = go ? e1r : 1.0f;
    const float w1 = T0 * (1.0f - e1);
    acc.C0 = __builtin_fmaf(w1, __builtin_fmaf(g1, db.x, b0.x), acc.C0);
    acc.C1 = __builtin_fmaf(w1, __builtin_fmaf(g1, db.y, b0.y), acc.C1);
    acc.C2 = __builtin_fmaf(w1, __builtin_fmaf(g1, db.z, b0.z), acc.C2);
    acc.T = T0 * e1;
    nexec += go ? 2u : 1u;
    return acc.T <= R.ert_T;
}

template <int MODE>
__device__ __forceinline__ void store_pixel(const DevReq& R, int px, int py, bool hit,
                                            const Accum& acc) {
    const int64_t pix = (int64_t)py * R.W + px;
    if (MODE == 0) {
        *(float4*)(R.out + 4 * pix) =
            hit ? make_float4(acc.C0, acc.C1, acc.C2, 1.0f - acc.T) : make_float4(0.f, 0.f, 0.f, 0.f);
    } else if (!R.partial) {
        R.out[pix] = hit ? ((acc.m >= R.tf.clip) ? acc.m * R.out_scale : 0.0f) : -VR_INF;
    } else {
        // sub-cube partial: -inf without samples in the window, the lowest
        // float where they all lie below the clip (combined by maximum, then
        // floored to 0)
        R.out[pix] = hit ? ((acc.m >= R.tf.clip) ? acc.m * R.out_scale : -3.402823466e38f) : -VR_INF;
    }
}

__device__ __forceinline__ void tile_pixel(const DevReq& R, int tx, int ty, int& px, int& py) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    px = tx * VR_TW + (wave % (VR_TW / 8)) * 8 + (lane & 7);
    py = ty * VR_TH + (wave / (VR_TW / 8)) * 8 + (lane >> 3);
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
    if (n == 0 || ray.kb >= ray.ke) {
        store_pixel<MODE>(R, px, py, false, acc);
        return;
    }
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    const int B[3] = {R.cube.bx, R.cube.by, R.cube.bz};
    float inv_dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) inv_dd[a] = ray.dd[a] != 0.0f ? 1.0f / ray.dd[a] : 0.0f;
    const float shift = INTERP == 0 ? 0.5f : 0.0f;
    int k0 = ray.kb, m = 0, j = 0;
    float A[3] = {0.0f, 0.0f, 0.0f}, hb[3] = {0.0f, 0.0f, 0.0f};
    const uint8_t* base = nullptr;
    uint64_t mask = 0;
    unsigned nexec = 0, nskip = 0;
    bool stopped = false;
    while (true) {
        if (j >= m) {
            k0 += m;
            if (k0 >= ray.ke) break;
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
            const int rem = ray.ke - k0;
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
        const float v = slot_value<DT, INTERP>((const VT*)base, R.cube.xch, i0, i1, i2, w0, w1, w2);
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
    cnt.nominal += (unsigned)(ray.ke - ray.kb);
    cnt.exec += nexec;
    cnt.hit += 1u;
    cnt.ert += stopped ? 1u : 0u;
    cnt.skipped += nskip;
}

// ---------------------------------------------------------------------------
// Slab-staged tile renderer (the main path).
//
// A workgroup (VR_WG threads, two per compute unit) owns a 16x16 pixel tile (one
// 8x8 block per wave) and marches all its rays in
// lock-step through slabs along the major axis M of the tile's view direction,
// front to back.  Every ray of the tile passes, at any plane perpendicular to
// M, inside the quadrilateral cut by the tile's four corner rays (the tile's
// rays form a pyramid, or a prism for orthographic views), so the box of voxel
// indices the samples of a slab can touch follows from the corner rays alone.
// Each slab is the thickest (up to 32 voxels, and at most twice the previous
// one) whose box fits twice a fixed reference size; that choice depends only
// on the tile's geometry, so the image never depends on staging decisions,
// batch composition or the LDS the caller leaves free.  The box's 8^3 cells
// are tested against the skip grid two slabs ahead, the next slab's box is
// copied into LDS with 16-byte global->LDS loads once the current slab has
// been sampled, and every lane interpolates its ray's samples of the slab
// from LDS, skipping runs of 8 samples whose cells are all inactive where few
// cells are active.  A box larger than its buffer is sampled straight from
// the brick pool with the same arithmetic.
// ---------------------------------------------------------------------------
#define VR_BIG 0x3fffffff
#define VR_SMAX 32


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

// Voxel index and weights of a position in box-local coordinates: clamped to
// [0, hi] (the cube's last voxel on the upper side; the box never starts below
// a sample), so truncation is the floor.  Trilinear at q = N - 1 takes the last
// voxel with weight 0 (its +1 neighbour is the edge-clamped apron).
template <int INTERP>
__device__ __forceinline__ void floor_idx(const float p[3], const float hi[3], int i[3], float w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = __builtin_amdgcn_fmed3f(p[a], 0.0f, hi[a]);
        if (INTERP == 1) {
            w[a] = __builtin_amdgcn_fractf(q);
            i[a] = (int)q;
        } else {
            w[a] = 0.0f;
            i[a] = (int)(q + 0.5f);
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

// The tile's corner rays as lines over the major axis: on the plane M = z the
// corner ray k sits at lateral coordinate c[k][q] + z * r[k][q] (q = 0 for axis
// (M+1)%3, 1 for (M+2)%3).
struct Corners {
    float c[4][2], r[4][2];
};

// LDS elements per z plane of a box: np chunks per row and d1 rows.  Rows
// start 16-byte aligned (odd np spreads them over the LDS banks four dwords
// apart).  When M is x, the lanes of a wave read at nearly the same x and
// differ in y and z, which leaves them few bank groups; one dword more per
// plane (global->LDS loads accept dword-aligned LDS addresses) spreads them
// over all banks.
template <int M, int CV>
__device__ __forceinline__ int box_skew() {
    return M == 0 ? CV / 4 : 0;
}
template <int M, int CV>
__device__ __forceinline__ int box_plane(int np, int d1) {
    return np * CV * d1 + box_skew<M, CV>();
}

// One slab: planes [z0, z0 + S] along M, and the box of voxel indices its
// samples can touch (floor indices plus the +1 neighbour), with floor indices
// clamped to [CL, CH] per axis: the cube, narrowed on a sub-cube window's axis
// to the planes its samples can touch.
struct Slab {
    int z0, S;
    int lo[3], dim[3];
    int xa, nc;   // first 16-byte-aligned x of the box, 16-byte chunks of data per box row
    int np;       // chunks per LDS row: nc, rounded up to odd from 3 chunks on so
                  // that consecutive rows start on different LDS banks
    int elems;    // LDS elements of the box (row pitch np * chunk), 0 if empty
    int big;      // the box takes both LDS buffers
    int boff;     // byte offset of the box in the LDS box area
    int late;     // copied only after the previous slab is sampled (it or the
                  // previous slab takes both buffers)
};

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// skip-grid rows of a slab box kept in LDS for the waves' own checks
#define VR_CROW 128

struct TileShared {
    int red[4];         // tile-start reductions: first/last sample planes
    int any[8];         // slab k may contribute (skip grid), ring by k % 8
    unsigned nact[8];   // active cells of slab k's box (2^20 and up: rows not kept), ring by k % 8
    int alive[3];       // some ray still marching after slab k, ring by k % 3
    Slab ring[4];       // slab k's geometry, ring by k % 4 (S == 0: no such slab)
    uint64_t crow[3][VR_CROW];  // slab k's cell rows (bit i: cell c0x + i), ring by k % 3
};

template <int M, int CV>
__device__ __forceinline__ Slab slab_box(int z0, int S, const Corners& cr, const int N[3],
                                         const int CL[3], const int CH[3], int zmin, int zmax) {
    constexpr int A1 = (M + 1) % 3, A2 = (M + 2) % 3;
    Slab s;
    s.z0 = z0;
    s.S = S;
    // samples of the slab lie on [z0, z0 + S] along M up to rounding; at the
    // cube's faces they can also lie in [-1/2, 0) or (N - 1, N - 1/2]
    float za = z0 <= 0 ? -0.5f : (float)z0;
    float zb = z0 + S >= N[M] - 1 ? (float)N[M] - 0.5f : (float)(z0 + S);
    za -= 1e-3f;
    zb += 1e-3f;
    int lo[3], hi[3];
    lo[M] = max(max(z0 - 1, zmin - 1), CL[M]);
    hi[M] = min(min(z0 + S, zmax + 1), CH[M]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a = q == 0 ? A1 : A2;
        float mn = VR_INF, mx = -VR_INF;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float v0 = __builtin_fmaf(za, cr.r[k][q], cr.c[k][q]);
            const float v1 = __builtin_fmaf(zb, cr.r[k][q], cr.c[k][q]);
            mn = fminf(mn, fminf(v0, v1));
            mx = fmaxf(mx, fmaxf(v0, v1));
        }
        // sample positions lie in [-1/2, N - 1/2] and their indices are those
        // of the position clamped to [0, N - 1]: a bundle that only reaches
        // the sliver [-1/2, 0) still reads voxel 0 (and [N - 1, N - 1/2] voxel N - 1)
        lo[a] = max((int)floorf(fminf(mn, (float)(N[a] - 1)) - 0.01f), CL[a]);
        hi[a] = min((int)floorf(fmaxf(mx, 0.0f) + 0.01f), CH[a]);
    }
    bool empty = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.lo[a] = lo[a];
        s.dim[a] = hi[a] - lo[a] + 2;
        empty = empty || hi[a] < lo[a];
    }
    s.xa = lo[0] & ~(CV - 1);
    s.nc = (lo[0] + s.dim[0] - 1 - s.xa) / CV + 1;
    s.np = s.nc >= 3 ? (s.nc | 1) : s.nc;
    s.big = 0;
    s.boff = 0;
    s.late = 0;
    s.elems = empty ? 0 : box_plane<M, CV>(s.np, s.dim[1]) * s.dim[2];
    return s;
}

// Thickest slab entered at plane ze, at most hi <= 64 voxels, whose box holds
// at most cap elements; ok = false when not even one voxel fits.  Called by a
// whole wave: lane l tries thickness l + 1, and as the box only grows with the
// thickness, the lanes that fit are exactly those below the answer.
template <int M, int CV>
__device__ __forceinline__ Slab fit_slab(int ze, int sgn, int hi, int cap, const Corners& cr,
                                         const int N[3], const int CL[3], const int CH[3],
                                         int zmin, int zmax, bool& ok) {
    const int t = min((int)(threadIdx.x & 63) + 1, hi);
    const Slab m = slab_box<M, CV>(sgn > 0 ? ze : ze - t, t, cr, N, CL, CH, zmin, zmax);
    const int S = min(__popcll(__ballot(m.elems <= cap)), hi);
    ok = S > 0;
    return slab_box<M, CV>(sgn > 0 ? ze : ze - max(S, 1), max(S, 1), cr, N, CL, CH, zmin, zmax);
}

// Next slab entered at plane ze: the thickest (at most twice the previous
// thickness and VR_SMAX) whose box fits both LDS buffers of the reference
// size.  Such a box is copied only after the slab before it has been sampled;
// measured on the full-size workload, slabs twice as thick beat overlapping
// the copy of a one-buffer box with the sampling of the previous slab.  A box
// that does not fit even one voxel thick is marched 8 voxels at a time from
// the brick pool.  Only geometry decides, never the LDS a launch actually has.
template <int M, int CV, int ELEM>
__device__ __forceinline__ Slab next_slab(int ze, int sgn, int Sprev, const Corners& cr,
                                          const int N[3], const int CL[3], const int CH[3],
                                          int zmin, int zmax) {
    constexpr int cap = VR_BOX_REF / ELEM;
    bool ok;
    Slab b = fit_slab<M, CV>(ze, sgn, min(VR_SMAX, 2 * Sprev), 2 * cap, cr, N, CL, CH, zmin, zmax, ok);
    if (ok) {
        b.big = 1;
        return b;
    }
    return slab_box<M, CV>(sgn > 0 ? ze : ze - 8, 8, cr, N, CL, CH, zmin, zmax);
}

// Anchor of lattice sample k0 (without the last segment's shift) relative to
// the integer point lo on one axis: E + (k0 + 1/2) step d - lo, with E the
// ray's entry point, evaluated in float-float and rounded once.
__device__ __forceinline__ float anchor_axis(const ff& E, const ff& d, const ff& sk, int lo) {
#pragma clang fp contract(off)
    ff h = two_sum(E.hi, -(float)lo);
    h.lo += E.lo;
    const ff p = ff_mul(sk, d);
    const ff q = two_sum(h.hi, p.hi);
    return q.hi + (q.lo + (h.lo + p.lo));
}

template <int MODE, int DT, int INTERP, int M>
__device__ __forceinline__ bool tile_march(const DevReq& R, const Ray& ray, const int px,
                                           const int py, const bool inimg, const Corners& cr,
                                           const int sgn, const float* __restrict__ tfl,
                                           uint8_t* __restrict__ boxes, TileShared& sh,
                                           LaneCounts& cnt) {
    typedef typename Vox<DT>::T VT;
    typedef __attribute__((address_space(3))) const VT LVT;
    constexpr int ELEM = DT == 0 ? 4 : 2;
    constexpr int CV = 16 / ELEM;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int N[3] = {R.cube.nx, R.cube.ny, R.cube.nz};
    int CL[3] = {0, 0, 0}, CH[3] = {N[0] - 1, N[1] - 1, N[2] - 1};
    if (R.win_axis >= 0) {
        const int a = R.win_axis;
        CL[a] = max(CL[a], R.win_vlo);
        CH[a] = min(CH[a], R.win_vhi - 1);
    }
    const int cap = R.box_bytes / ELEM;
    const bool act = ray.n > 0 && ray.kb < ray.ke;

    // ---- tile-wide range of sample planes along M -----------------------------
    int zf = 0, zl = 0;
    ff E[3];
    if (act) {
        const ff t1 = sample_t(R, ray, ray.ke - 1);
        const ff t0 = sample_t(R, ray, ray.kb);
#pragma unroll
        for (int a = 0; a < 3; ++a) E[a] = ff_add(ray.o[a], ff_mul(ray.tin, ray.d[a]));
        const float pf = ff_to_f(ff_add(ray.o[M], ff_mul(t0, ray.d[M])));
        const float pl = ff_to_f(ff_add(ray.o[M], ff_mul(t1, ray.d[M])));
        const float hm = (float)(N[M] - 1);
        zf = (int)floorf(fminf(fmaxf(pf, 0.0f), hm));
        zl = (int)floorf(fminf(fmaxf(pl, 0.0f), hm));
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) E[a] = ff_make(0.0f);
    }
    {
        const int a = wave_min(act ? min(zf, zl) : VR_BIG);
        const int b = wave_max(act ? max(zf, zl) : -VR_BIG);
        if (lane == 0) {
            atomicMin(&sh.red[0], a);
            atomicMax(&sh.red[1], b);
        }
    }
    __syncthreads();
    int zmin = sh.red[0], zmax = sh.red[1];
    if (zmin == VR_BIG) {  // no ray of the tile meets the cube: no slab
        zmin = 0;
        zmax = -1;
    }
    // planes: marching up, slabs start at zmin and go while the entry plane is
    // <= zmax; marching down, they start at zmax + 1 and go while entry > zmin
    auto slab_exists = [&](int ze) { return sgn > 0 ? ze <= zmax : ze > zmin; };
    auto exit_plane = [&](const Slab& s) { return sgn > 0 ? s.z0 + s.S : s.z0; };
    // wave 0 lays out the slabs (identical in every lane) and publishes them
    // Buffers: a one-buffer box goes to the buffer the previous slab does not
    // use; a two-buffer box, and any box after one, is copied late.
    Slab w0 = {};
    bool w0_first = true;
    int w0_buf = 1;
    auto produce = [&](int slot) {
        Slab s = {};
        if (w0_first) {
            const int ze = sgn > 0 ? zmin : zmax + 1;
            if (slab_exists(ze)) s = next_slab<M, CV, ELEM>(ze, sgn, VR_SMAX, cr, N, CL, CH, zmin, zmax);
        } else if (w0.S != 0 && slab_exists(exit_plane(w0))) {
            s = next_slab<M, CV, ELEM>(exit_plane(w0), sgn, w0.S, cr, N, CL, CH, zmin, zmax);
        }
        if (s.S != 0) {
            const int buf = (s.big || w0.big) ? 0 : 1 - w0_buf;
            s.boff = buf * R.box_bytes;
            s.late = (!w0_first && (s.big || w0.big)) ? 1 : 0;
            w0_buf = buf;
        }
        w0_first = false;
        if (lane == 0) sh.ring[slot] = s;
        w0 = s;
    };

    // ---- per-ray state --------------------------------------------------------------
    const float om = act ? ff_to_f(ray.o[M]) : 0.0f;
    const float inv_dm = act ? 1.0f / ray.d[M].hi : 0.0f;
    const float tinf = act ? ff_to_f(ray.tin) : 0.0f;
    const float inv_step = 1.0f / ff_to_f(R.step);
    Accum acc = {0.0f, 0.0f, 0.0f, 1.0f, -VR_INF};
    unsigned nexec = 0, nskip = 0;
    bool stopped = false;
    // first sample past the exit plane of a slab
    auto slab_end = [&](const Slab& s, int kprev) -> int {
        if (!act || stopped || s.S == 0) return kprev;
        const int zx = exit_plane(s);
        if (sgn > 0 ? zx > zl : zx <= zl) return ray.ke;
        const float kf = ceilf((((float)zx - om) * inv_dm - tinf) * inv_step - 0.5f);
        return kf < (float)kprev ? kprev : (kf > (float)ray.ke ? ray.ke : (int)kf);
    };
    // Skip-grid words of a slab's cells: bits_issue loads them (one row of cells
    // along x per thread); bits_done, once they have landed, marks the slab as
    // possibly contributing and keeps rows of up to 64 cells in LDS (slabs of at
    // most VR_CROW rows) for the finer per-wave checks during sampling.
    const int Cx = 4 * R.cube.bx, Cy = 4 * R.cube.by;
    struct Bits {
        uint32_t w0, w1, m0, m1;
        int lob, row;  // first bit in word w0; LDS row this thread keeps (-1: none)
        int wide;      // treated as active; the slab's rows are not kept
        int nofine;    // the slab's rows are not kept
    };
    auto bits_issue = [&](const Slab& s) -> Bits {
        Bits b = {0u, 0u, 0u, 0u, 0, -1, 0, 0};
        if (s.S == 0 || s.elems == 0) return b;
        int c0[3], c1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c0[a] = s.lo[a] >> 3;
            c1[a] = (s.lo[a] + s.dim[a] - 2) >> 3;
        }
        const int ny_ = c1[1] - c0[1] + 1, nrow = ny_ * (c1[2] - c0[2] + 1);
        if (nrow > VR_WG) {
            b.wide = tid == 0;  // more cell rows than threads: treated as active
            return b;
        }
        b.nofine = (tid == 0 && nrow > VR_CROW) ? 1 : 0;
        if (tid >= nrow) return b;
        const int czr = div_small(tid, ny_, 1.0f / (float)ny_);
        const int cy = c0[1] + tid - czr * ny_, cz = c0[2] + czr;
        const int64_t b0 = ((int64_t)cz * Cy + cy) * Cx + c0[0];
        const int64_t b1 = b0 + (c1[0] - c0[0]);
        const int64_t wa = b0 >> 5, wb = b1 >> 5;
        if (wb - wa > 1) {
            b.wide = 1;  // more than two words: treated as active
            return b;
        }
        const uint32_t lo_bit = (uint32_t)(b0 & 31), hi_bit = (uint32_t)(b1 & 31);
        if (wa == wb) {
            b.m0 = (hi_bit == 31 ? 0xffffffffu : ((1u << (hi_bit + 1)) - 1u)) & ~((1u << lo_bit) - 1u);
        } else {
            b.m0 = ~((1u << lo_bit) - 1u);
            b.m1 = hi_bit == 31 ? 0xffffffffu : ((1u << (hi_bit + 1)) - 1u);
            b.w1 = R.cube.cellbits[wb];
        }
        b.w0 = R.cube.cellbits[wa];
        b.lob = (int)lo_bit;
        b.row = nrow <= VR_CROW ? tid : -1;
        return b;
    };
    auto bits_done = [&](int k, const Bits& b) {
        const uint32_t lo = b.w0 & b.m0, hi = b.w1 & b.m1;
        if (b.wide || lo || hi) sh.any[k & 7] = 1;
        unsigned add = (b.wide || b.nofine) ? (1u << 20) : 0u;
        if (b.row >= 0) {
            const uint64_t r = ((((uint64_t)hi) << 32) | lo) >> b.lob;
            sh.crow[k % 3][b.row] = r;
            add += (unsigned)__popcll(r);
        }
        if (add) atomicAdd(&sh.nact[k & 7], add);
    };
    // MIP running-maximum skipping: the bound of each of the box's 8^3 cells
    // (DevCube::cellmax) is kept in LDS, three slabs in flight like the cell
    // rows, copied two slabs ahead with 4-byte global->LDS loads (lane l of a
    // wave instruction copies cell f0 + l of the box's cells in row order).
    // Boxes with rows longer than VR_TROW cells or more than VR_MIPC cells are
    // sampled without it.
    float* const cthr = MODE == 1 ? const_cast<float*>(tfl) : nullptr;
    auto thr_ok = [&](const Slab& s) -> bool {
        if (MODE != 1 || !R.use_skip || !R.cube.cellmax || s.S == 0 || s.elems == 0) return false;
        const int nxc = ((s.lo[0] + s.dim[0] - 2) >> 3) - (s.lo[0] >> 3) + 1;
        const int nyc = ((s.lo[1] + s.dim[1] - 2) >> 3) - (s.lo[1] >> 3) + 1;
        const int nzc = ((s.lo[2] + s.dim[2] - 2) >> 3) - (s.lo[2] >> 3) + 1;
        return nxc <= VR_TROW && nxc * nyc * nzc <= VR_MIPC;
    };
    // where more than half of a box's cells can reach the clip, the bounds
    // rarely let a chunk pass and are not used (nor copied)
    auto thr_use = [&](const Slab& s, int k) -> bool {
        if (MODE != 1 || !thr_ok(s)) return false;
        const int nc = (((s.lo[0] + s.dim[0] - 2) >> 3) - (s.lo[0] >> 3) + 1) *
                       (((s.lo[1] + s.dim[1] - 2) >> 3) - (s.lo[1] >> 3) + 1) *
                       (((s.lo[2] + s.dim[2] - 2) >> 3) - (s.lo[2] >> 3) + 1);
        return 2u * (unsigned)__builtin_amdgcn_readfirstlane((int)sh.nact[k & 7]) <= (unsigned)nc;
    };
    auto thr_dma = [&](const Slab& s, int k) {
        if (MODE != 1 || !thr_use(s, k)) return;
        const int c0x = s.lo[0] >> 3, c0y = s.lo[1] >> 3, c0z = s.lo[2] >> 3;
        const int nxc = ((s.lo[0] + s.dim[0] - 2) >> 3) - c0x + 1;
        const int nyc = ((s.lo[1] + s.dim[1] - 2) >> 3) - c0y + 1;
        const int ncell = nxc * nyc * (((s.lo[2] + s.dim[2] - 2) >> 3) - c0z + 1);
        const float inv_x = 1.0f / (float)nxc, inv_y = 1.0f / (float)nyc;
        float* dst = cthr + (k % 3) * VR_MIPC;
        for (int f0 = wave * 64; f0 < ncell; f0 += VR_NWAVE * 64) {
            const int f = f0 + lane;
            if (f < ncell) {
                const int row = div_small(f, nxc, inv_x), col = f - row * nxc;
                const int czr = div_small(row, nyc, inv_y), cyr = row - czr * nyc;
                const int64_t g = ((int64_t)(c0z + czr) * Cy + (c0y + cyr)) * Cx + c0x + col;
                __builtin_amdgcn_global_load_lds((const void*)(R.cube.cellmax + g),
                                                 (__attribute__((address_space(3))) void*)(dst + f0),
                                                 4, 0, 0);
            }
        }
    };
    // Copy a slab's box into its LDS buffer: the box is row-major over
    // [z][y][16-byte chunk] with np chunks per row and planes box_plane()
    // elements apart, and global->LDS loads write 16 bytes per lane at
    // consecutive LDS addresses, so each wave instruction moves rw = 64 / np
    // whole rows of one plane (lane l: row l / np, chunk l % np).  A voxel's
    // pool address is the sum of a part that depends on its z only (the layer
    // of bricks and the plane inside the slot) and a part that depends on its
    // y and x only, so each lane computes its y/x part once per group of rows
    // and the waves walk the planes with the z part alone (wave-uniform).
    // Rows of more than 64 chunks go one row per instruction group.
    auto staged = [&](const Slab& s) { return s.elems <= (s.big ? 2 * cap : cap); };
    const uint32_t bstride = (uint32_t)R.cube.stride;
    auto row_src = [&](const Slab& s, int iy, int iz) -> const uint8_t* {
        const int gy = min(s.lo[1] + iy, N[1] - 1), gz = min(s.lo[2] + iz, N[2] - 1);
        const int bzl = min(gz >> 5, R.cube.bz_hi - 1);  // plane 32 of a layer: its apron
        const uint32_t slot_yz = __umul24(__umul24(bzl, R.cube.by) + (gy >> 5), R.cube.bx);
        const uint32_t off = (uint32_t)(slot_y<DT>(gy & 31, R.cube.xch) + slot_z<DT>(gz - 32 * bzl, R.cube.xch)) * ELEM;
        return R.cube.pool + ((uint64_t)slot_yz * bstride + off);
    };
    auto chunk_off = [&](const Slab& s, int c) -> uint64_t {
        const int x = s.xa + min(c, s.nc - 1) * CV;  // pad slots repeat the last chunk
        const int bxb = min(x >> 5, R.cube.bx - 1);
        return (uint64_t)bxb * bstride + (uint32_t)(((x - 32 * bxb) / CV) * 128);
    };
    auto box_dma = [&](const Slab& s) {
        if (s.S == 0 || s.elems == 0 || !staged(s)) return;
        uint8_t* buf = boxes + s.boff;
        const int np = s.np, d1 = s.dim[1], d2 = s.dim[2];
        const int plane_bytes = box_plane<M, CV>(np, d1) * ELEM;
        const uint64_t layer = (uint64_t)R.cube.by * R.cube.bx * bstride;  // bytes of a layer of bricks
        if (np <= 64) {
            const int lo1 = __builtin_amdgcn_readfirstlane(s.lo[1]);
            const int lo2 = __builtin_amdgcn_readfirstlane(s.lo[2]);
            const int u1 = __builtin_amdgcn_readfirstlane(d1), u2 = __builtin_amdgcn_readfirstlane(d2);
            const int unp = __builtin_amdgcn_readfirstlane(np);
            const int upb = __builtin_amdgcn_readfirstlane(plane_bytes);
            const int wv = __builtin_amdgcn_readfirstlane(wave);
            uint8_t* const ubuf = boxes + __builtin_amdgcn_readfirstlane(s.boff);
            const float inv_np = 1.0f / (float)unp;
            const int rw = div_small(64, unp, inv_np);
            const int lr = div_small(lane, unp, inv_np);
            const uint64_t xo = chunk_off(s, lane - lr * unp);
            const uint64_t brow = (uint64_t)R.cube.bx * bstride;  // bytes of a row of bricks
            auto zpart = [&](int iz) -> uint64_t {
                const int gz = min(lo2 + iz, N[2] - 1);
                const int bzl = min(gz >> 5, R.cube.bz_hi - 1);  // plane 32 of a layer: its apron
                return (uint64_t)R.cube.pool + (uint64_t)bzl * layer +
                       (uint32_t)slot_z<DT>(gz - 32 * bzl, R.cube.xch) * ELEM;
            };
            // z parts of this wave's planes wv + 4k, one per lane k, read back
            // with readlane (for boxes of at most 256 planes)
            const bool ztab = u2 <= VR_NWAVE * 64;
            const uint64_t zv = ztab && wv + VR_NWAVE * lane < u2 ? zpart(wv + VR_NWAVE * lane) : 0ull;
            const uint32_t zv_lo = (uint32_t)zv, zv_hi = (uint32_t)(zv >> 32);
            for (int y0 = 0; y0 < u1; y0 += rw) {
                const int gy = min(lo1 + y0 + lr, N[1] - 1);
                uint64_t yx = (uint64_t)(gy >> 5) * brow + (uint32_t)slot_y<DT>(gy & 31, R.cube.xch) * ELEM + xo;
                asm volatile("" : "+v"(yx));  // one register pair, not re-summed per plane
                const bool on = lr < rw && y0 + lr < u1;
                for (int iz = wv, k = 0; iz < u2; iz += VR_NWAVE, ++k) {
                    const uint64_t zp =
                        ztab ? ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)zv_hi, k) << 32) |
                                   (uint32_t)__builtin_amdgcn_readlane((int)zv_lo, k)
                             : zpart(iz);
                    if (on)
                        __builtin_amdgcn_global_load_lds((const void*)(zp + yx),
                                                         (__attribute__((address_space(3))) void*)(ubuf + iz * upb + y0 * unp * 16),
                                                         16, 0, 0);
                }
            }
            return;
        }
        const int rows = d1 * d2;
        const float inv_d1 = 1.0f / (float)d1;
        for (int r = wave; r < rows; r += VR_NWAVE) {
            const int iz = div_small(r, d1, inv_d1), iy = r - iz * d1;
            const uint8_t* src = row_src(s, iy, iz);
            for (int c0 = 0; c0 < np; c0 += 64) {
                if (c0 + lane < np)
                    __builtin_amdgcn_global_load_lds((const void*)(src + chunk_off(s, c0 + lane)),
                                                     (__attribute__((address_space(3))) void*)(buf + iz * plane_bytes + (iy * np + c0) * 16),
                                                     16, 0, 0);
            }
        }
    };


    // ---- prologue: slabs 0 and 1 ------------------------------------------------------
    if (wave == 0) {
        produce(0);
        produce(1);
    }
    __syncthreads();
    Slab s0 = sh.ring[0], s1 = sh.ring[1];
    int ks = act ? ray.kb : 0, ke0 = slab_end(s0, ks);
    if (R.use_skip) {
        bits_done(0, bits_issue(s0));
        bits_done(1, bits_issue(s1));
        __syncthreads();
        thr_dma(s0, 0);
    }
    if (sh.any[0]) box_dma(s0);

    // ---- slab pipeline -----------------------------------------------------------------
    for (int it = 0; s0.S != 0; ++it) {
        if (wave == 0) produce((it + 2) & 3);
        if (tid == 0) {
            sh.any[(it + 3) & 7] = R.use_skip ? 0 : 1;
            sh.nact[(it + 3) & 7] = 0u;
            sh.alive[it % 3] = 0;
        }
        __builtin_amdgcn_s_waitcnt(0);  // own box copies of slab it have landed
        __syncthreads();
        if (it > 0 && sh.alive[(it - 1) % 3] == 0) break;
        const Slab s2 = sh.ring[(it + 2) & 3];
        Bits bb = {0u, 0u, 0u, 0u, 0, -1, 0, 0};
        if (R.use_skip) bb = bits_issue(s2);
        thr_dma(s1, it + 1);  // its ring entry held slab it - 2; lands by the next iteration
        if (!s1.late && sh.any[(it + 1) & 7]) box_dma(s1);
        const int ke1 = slab_end(s1, ke0);
        // MIP: passing over samples that cannot raise the running maximum.  A
        // wave checks its chunks only where at most a quarter of the box's
        // cells could raise the smallest running maximum among its rays still
        // marching (otherwise the checks would cost more than they save).
        bool use_thr = MODE == 1 && thr_use(s0, it);
        if (MODE == 1 && use_thr) {
            float mlo = act && !stopped && ks < ray.ke ? acc.m : VR_INF;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mlo = fminf(mlo, __shfl_xor(mlo, o));
            const float* cth0 = cthr + (it % 3) * VR_MIPC;
            const int nc = (((s0.lo[0] + s0.dim[0] - 2) >> 3) - (s0.lo[0] >> 3) + 1) *
                           (((s0.lo[1] + s0.dim[1] - 2) >> 3) - (s0.lo[1] >> 3) + 1) *
                           (((s0.lo[2] + s0.dim[2] - 2) >> 3) - (s0.lo[2] >> 3) + 1);
            int above = 0;
            for (int f = lane; f - lane < nc; f += 64)
                above += __popcll(__ballot(f < nc && cth0[f] > mlo));
            use_thr = 4 * above <= nc;
        }
        // ---- sample slab it
        const int cnt_s = ke0 - ks;
        if (cnt_s > 0 && !stopped) {
            if (!sh.any[it & 7]) {
                nskip += (unsigned)cnt_s;
            } else {
                float A[3], ch[3];
                {
                    const float kf = (float)ks + 0.5f;
                    ff sk = two_prod(kf, R.step.hi);
                    sk.lo = __builtin_fmaf(kf, R.step.lo, sk.lo);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        A[a] = anchor_axis(E[a], ray.d[a], sk, s0.lo[a]);
                        ch[a] = (float)(N[a] - 1 - s0.lo[a]);
                    }
                }
                // samples are taken two at a time so that the second one's box
                // reads are in flight while the first one is classified
                auto value = [&](auto fetch, int j, bool last) {
                    const float jf = (float)j + (last ? ray.last_adj : 0.0f);
                    const float p[3] = {__builtin_fmaf(jf, ray.dd[0], A[0]),
                                        __builtin_fmaf(jf, ray.dd[1], A[1]),
                                        __builtin_fmaf(jf, ray.dd[2], A[2])};
                    int i[3];
                    float w[3];
                    floor_idx<INTERP>(p, ch, i, w);
                    return fetch(i, w);
                };
                // Finer skip where under a quarter of the box's cells are
                // active: before every 8 samples each lane bounds the cells
                // its samples j .. j+7 can touch (positions at j - 1/2, the
                // last sample's earliest, and j + 7: per axis the clamped
                // index is monotone in the position), and the wave passes
                // over the 8 samples when no lane touches an active cell.
                int cb0[3], cb1[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    cb0[a] = s0.lo[a] >> 3;
                    cb1[a] = (s0.lo[a] + s0.dim[a] - 2) >> 3;
                }
                const int nyc = cb1[1] - cb0[1] + 1;
                const unsigned ncell = (unsigned)((cb1[0] - cb0[0] + 1) * nyc * (cb1[2] - cb0[2] + 1));
                const bool fine = use_thr || (R.use_skip && 4u * (unsigned)__builtin_amdgcn_readfirstlane((int)sh.nact[it & 7]) <= ncell);
                const uint64_t* crow = sh.crow[it % 3];
                auto live = [&](int j) -> bool {
                    const float ja = (float)j - 0.5f, jb = (float)j + 7.0f;
                    int c_lo[3], c_hi[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float qa = __builtin_amdgcn_fmed3f(__builtin_fmaf(ja, ray.dd[a], A[a]), 0.0f, ch[a]);
                        const float qb = __builtin_amdgcn_fmed3f(__builtin_fmaf(jb, ray.dd[a], A[a]), 0.0f, ch[a]);
                        const int ia = INTERP == 1 ? (int)qa : (int)(qa + 0.5f);
                        const int ib = INTERP == 1 ? (int)qb : (int)(qb + 0.5f);
                        c_lo[a] = min(max((s0.lo[a] + min(ia, ib)) >> 3, cb0[a]), cb1[a]);
                        c_hi[a] = min(max((s0.lo[a] + max(ia, ib)) >> 3, cb0[a]), cb1[a]);
                    }
                    const int nbx = c_hi[0] - c_lo[0] + 1;
                    const uint64_t xm = (nbx >= 64 ? ~0ull : ((1ull << nbx) - 1ull)) << (c_lo[0] - cb0[0]);
                    uint64_t hit = 0;
                    for (int cz = c_lo[2]; cz <= c_hi[2]; ++cz)
                        for (int cy = c_lo[1]; cy <= c_hi[1]; ++cy)
                            hit |= crow[(cz - cb0[2]) * nyc + (cy - cb0[1])];
                    return (hit & xm) != 0ull;
                };
                // MIP: some cell the samples j .. j+7 can touch has a bound above
                // the running maximum (bounds are -inf for cells below the clip)
                const int nxc = cb1[0] - cb0[0] + 1;
                const float* cth = MODE == 1 ? cthr + (it % 3) * VR_MIPC : nullptr;
                auto live_max = [&](int j) -> bool {
                    const float ja = (float)j - 0.5f, jb = (float)j + 7.0f;
                    int c_lo[3], c_hi[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float qa = __builtin_amdgcn_fmed3f(__builtin_fmaf(ja, ray.dd[a], A[a]), 0.0f, ch[a]);
                        const float qb = __builtin_amdgcn_fmed3f(__builtin_fmaf(jb, ray.dd[a], A[a]), 0.0f, ch[a]);
                        const int ia = INTERP == 1 ? (int)qa : (int)(qa + 0.5f);
                        const int ib = INTERP == 1 ? (int)qb : (int)(qb + 0.5f);
                        c_lo[a] = min(max((s0.lo[a] + min(ia, ib)) >> 3, cb0[a]), cb1[a]) - cb0[a];
                        c_hi[a] = min(max((s0.lo[a] + max(ia, ib)) >> 3, cb0[a]), cb1[a]) - cb0[a];
                    }
                    float t = -VR_INF;
                    for (int cz = c_lo[2]; cz <= c_hi[2]; ++cz)
                        for (int cy = c_lo[1]; cy <= c_hi[1]; ++cy) {
                            const float* rowp = cth + (cz * nyc + cy) * nxc;
                            for (int cx = c_lo[0]; cx <= c_hi[0]; ++cx) t = fmaxf(t, rowp[cx]);
                        }
                    return t > acc.m;
                };
                auto run = [&](auto fetch, auto fetch2, auto chunked) {
                    const int jl = ray.n - 1 - ks;  // index of the ray's last sample in this slab, if any
                    int j = 0;
                    for (; j + 1 < cnt_s; j += 2) {
                        if (decltype(chunked)::value && (j & 7) == 0 &&
                            __ballot(MODE == 1 && use_thr ? live_max(j) : live(j)) == 0ull) {
                            nskip += (unsigned)min(8, cnt_s - j);
                            j += 6;
                            continue;
                        }
                        float v0, v1;
                        {
                            const float ja = (float)j, jb = (float)(j + 1) + (j + 1 == jl ? ray.last_adj : 0.0f);
                            const float pa[3] = {__builtin_fmaf(ja, ray.dd[0], A[0]),
                                                 __builtin_fmaf(ja, ray.dd[1], A[1]),
                                                 __builtin_fmaf(ja, ray.dd[2], A[2])};
                            const float pb[3] = {__builtin_fmaf(jb, ray.dd[0], A[0]),
                                                 __builtin_fmaf(jb, ray.dd[1], A[1]),
                                                 __builtin_fmaf(jb, ray.dd[2], A[2])};
                            int ia[3], ib[3];
                            float wa[3], wb[3];
                            floor_idx<INTERP>(pa, ch, ia, wa);
                            floor_idx<INTERP>(pb, ch, ib, wb);
                            fetch2(ia, wa, ib, wb, v0, v1);
                        }
                        if (MODE == 1) {
                            nexec += 2;
                            acc.m = fmaxf(acc.m, fmaxf(v0, v1));
                        } else if (composite2(R, tfl, v0, v1, j + 1 == jl, ray, acc, nexec)) {
                            stopped = true;
                            break;
                        }
                    }
                    if (j < cnt_s && !stopped) {
                        const float v = value(fetch, j, j == jl);
                        ++nexec;
                        if (MODE == 1) {
                            acc.m = fmaxf(acc.m, v);
                        } else if (composite(R, tfl, v, j == jl, ray, acc)) {
                            stopped = true;
                        }
                    }
                };
                if (staged(s0)) {
                    const LVT* box = (const LVT*)(boxes + s0.boff);
                    const int pitch = s0.np * CV;
                    const int sy = pitch, sz = box_plane<M, CV>(s0.np, s0.dim[1]);
                    const int xoff = s0.lo[0] - s0.xa;
                    // consecutive samples of a ray often share their cell: its
                    // corners are read from LDS only when the cell changes (a
                    // nearest sample's single read is cheaper than the test)
                    int cidx = -1;
                    float cc[8];
                    auto fetch = [&](const int* i, const float* w) {
                        const int idx = (int)__umul24(__umul24(i[2], s0.dim[1]) + i[1], pitch) + i[0] + xoff +
                                        i[2] * box_skew<M, CV>();
                        if (INTERP == 0) return Vox<DT>::dec(box[idx]);
                        if (idx != cidx) {
                            box_corners<DT>(box, idx, sy, sz, cc);
                            cidx = idx;
                        }
                        return trilerp(cc[0], cc[1], cc[2], cc[3], cc[4], cc[5], cc[6], cc[7], w[0], w[1], w[2]);
                    };
                    // two samples at once: both corner sets are read with one wait
                    auto fetch2 = [&](const int* ia, const float* wa, const int* ib, const float* wb,
                                      float& va, float& vb) {
                        const int sk = box_skew<M, CV>();
                        const int ja = (int)__umul24(__umul24(ia[2], s0.dim[1]) + ia[1], pitch) + ia[0] + xoff + ia[2] * sk;
                        const int jb = (int)__umul24(__umul24(ib[2], s0.dim[1]) + ib[1], pitch) + ib[0] + xoff + ib[2] * sk;
                        if (INTERP == 0) {
                            va = Vox<DT>::dec(box[ja]);
                            vb = Vox<DT>::dec(box[jb]);
                            return;
                        }
                        float ca[8], cb[8];
                        box_corners<DT>(box, ja, sy, sz, ca);
                        box_corners<DT>(box, jb, sy, sz, cb);
                        va = trilerp(ca[0], ca[1], ca[2], ca[3], ca[4], ca[5], ca[6], ca[7], wa[0], wa[1], wa[2]);
                        vb = trilerp(cb[0], cb[1], cb[2], cb[3], cb[4], cb[5], cb[6], cb[7], wb[0], wb[1], wb[2]);
                    };
                    if (fine)
                        run(fetch, fetch2, BoolC<true>());
                    else
                        run(fetch, fetch2, BoolC<false>());
                } else {
                    auto fetch = [&](const int* i, const float* w) {
                        return pool_value<DT, INTERP>(R.cube, s0.lo[0] + i[0], s0.lo[1] + i[1],
                                                      s0.lo[2] + i[2], w[0], w[1], w[2]);
                    };
                    auto fetch2 = [&](const int* ia, const float* wa, const int* ib, const float* wb,
                                      float& va, float& vb) {
                        va = fetch(ia, wa);
                        vb = fetch(ib, wb);
                    };
                    if (fine)
                        run(fetch, fetch2, BoolC<true>());
                    else
                        run(fetch, fetch2, BoolC<false>());
                }
            }
        }
        if (R.use_skip) bits_done(it + 2, bb);
        const bool done = !act || stopped || ke0 >= ray.ke;
        if (__ballot(!done) != 0ull && lane == 0) sh.alive[it % 3] = 1;
        if (s1.late) {  // the box of slab it + 1 needs the LDS slab it used
            __syncthreads();
            if (sh.any[(it + 1) & 7]) box_dma(s1);
        }
        ks = ke0;
        ke0 = ke1;
        s0 = s1;
        s1 = s2;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (inimg) store_pixel<MODE>(R, px, py, act, acc);
    if (act) {
        cnt.nominal += (unsigned)(ray.ke - ray.kb);
        cnt.exec += nexec;
        cnt.hit += 1u;
        cnt.ert += stopped ? 1u : 0u;
        cnt.skipped += nskip;
    }
    return true;
}

// Returns false (having rendered nothing) when the rays of the tile do not all
// advance along one axis; the caller then runs the per-ray walker.
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
        for (int q = 0; q < 8; ++q) {
            sh.any[q] = R.use_skip ? 0 : 1;
            sh.nact[q] = 0u;
        }
        sh.alive[0] = sh.alive[1] = sh.alive[2] = 0;
    }
    // tile centre ray fixes the major axis; the corner rays bound the tile's
    // rays.  Lane k < 5 of each wave builds ray k (corners 0..3, centre 4) and
    // the values are broadcast, so the tile's geometry lives in scalar registers.
    const int lane = tid & 63, k5 = lane % 5;
    float o3[3], d3[3];
    {
        const float fi = k5 == 4 ? (float)(tx * VR_TW) + 0.5f * VR_TW
                                 : ((k5 & 1) ? (float)min(tx * VR_TW + VR_TW, R.W) - 0.5f : (float)(tx * VR_TW) + 0.5f);
        const float fj = k5 == 4 ? (float)(ty * VR_TH) + 0.5f * VR_TH
                                 : ((k5 & 2) ? (float)min(ty * VR_TH + VR_TH, R.H) - 0.5f : (float)(ty * VR_TH) + 0.5f);
        ff o[3], d[3];
        ray_dir(R.cam, fi, fj, o, d);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o3[a] = ff_to_f(o[a]);
            d3[a] = d[a].hi;
        }
    }
    auto bcast = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
    const float dc0 = bcast(d3[0], 4), dc1 = bcast(d3[1], 4), dc2 = bcast(d3[2], 4);
    const float ad0 = fabsf(dc0), ad1 = fabsf(dc1), ad2 = fabsf(dc2);
    const int m = (ad2 > ad0 && ad2 > ad1) ? 2 : (ad1 > ad0 ? 1 : 0);
    const float dm = m == 0 ? dc0 : (m == 1 ? dc1 : dc2);
    const int sgn = dm > 0.0f ? 1 : -1;
    const int m1 = m == 2 ? 0 : m + 1, m2 = m == 0 ? 2 : m - 1;
    const float dmk = m == 0 ? d3[0] : (m == 1 ? d3[1] : d3[2]);
    const float omk = m == 0 ? o3[0] : (m == 1 ? o3[1] : o3[2]);
    const float r1 = (m1 == 0 ? d3[0] : (m1 == 1 ? d3[1] : d3[2])) / dmk;
    const float r2 = (m2 == 0 ? d3[0] : (m2 == 1 ? d3[1] : d3[2])) / dmk;
    const float c1 = (m1 == 0 ? o3[0] : (m1 == 1 ? o3[1] : o3[2])) - omk * r1;
    const float c2 = (m2 == 0 ? o3[0] : (m2 == 1 ? o3[1] : o3[2])) - omk * r2;
    const bool ok = (__ballot(k5 < 4 && lane < 5 && (float)sgn * dmk >= 0.25f) & 0xfull) == 0xfull;
    Corners cr;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cr.r[k][0] = bcast(r1, k);
        cr.r[k][1] = bcast(r2, k);
        cr.c[k][0] = bcast(c1, k);
        cr.c[k][1] = bcast(c2, k);
    }
    if (!ok) return false;
    Ray ray;
    ray.n = 0;
    if (inimg) ray_setup(R, px, py, ray);
    __syncthreads();
    if (m == 0)
        return tile_march<MODE, DT, INTERP, 0>(R, ray, px, py, inimg, cr, sgn, tfl, boxes, sh, cnt);
    if (m == 1)
        return tile_march<MODE, DT, INTERP, 1>(R, ray, px, py, inimg, cr, sgn, tfl, boxes, sh, cnt);
    return tile_march<MODE, DT, INTERP, 2>(R, ray, px, py, inimg, cr, sgn, tfl, boxes, sh, cnt);
}

// One tile: slab-staged if possible, else one independent walker per ray.
template <int MODE, int DT, int INTERP>
__device__ __forceinline__ void render_tile_any(const DevReq& R, const int tx, const int ty,
                                                const float* __restrict__ tfl,
                                                uint8_t* __restrict__ boxes, TileShared& sh,
                                                LaneCounts& cnt) {
    if (render_tile<MODE, DT, INTERP>(R, tx, ty, tfl, boxes, sh, cnt)) return;
    __builtin_amdgcn_s_waitcnt(0);  // transfer-function rows have landed
    __syncthreads();
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

// Transfer-function rows (n x 32 bytes) copied into LDS with global->LDS loads
// (16 bytes per lane at consecutive LDS addresses).  Nothing waits for them
// here: the first slab's wait for its box copy (or the fallback walker's wait)
// covers them, so their latency overlaps the tile's set-up.
__device__ __forceinline__ void tf_stage(const DevReq& R, float4* lds4) {
    const float4* rows = (const float4*)R.tf.rows;
    for (int e = threadIdx.x; e < 2 * R.tf.n; e += VR_WG)
        __builtin_amdgcn_global_load_lds((const void*)(rows + e),
                                         (__attribute__((address_space(3))) void*)(lds4 + e), 16, 0, 0);
}

// dynamic LDS: transfer-function rows (n x 32 bytes), then two slab boxes
template <int MODE, int DT, int INTERP>
__global__ __launch_bounds__(VR_WG, VR_WAVES_PER_EU) void k_render(const DevReq R, const int* __restrict__ order,
                                                   DevCounters* cnt) {
    extern __shared__ float4 lds4[];
    __shared__ unsigned wgc[5];
    __shared__ TileShared sh;
    float* tfl = (float*)lds4;
    // EA: transfer-function rows; MIP: cell bounds of running-maximum skipping
    const int tf_bytes = MODE == 0 ? 32 * R.tf.n : VR_MIPC_BYTES;
    if (MODE == 0) tf_stage(R, lds4);
    if (cnt && threadIdx.x < 5) wgc[threadIdx.x] = 0u;
    __syncthreads();
    const int tile = order[blockIdx.x];
    const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
    LaneCounts c = {0u, 0u, 0u, 0u, 0u};
    render_tile_any<MODE, DT, INTERP>(R, tx, ty, tfl, (uint8_t*)lds4 + tf_bytes, sh, c);
    if (cnt) flush_counts(c, cnt, wgc);
}


// Static plus dynamic LDS of a launch must fit the compute unit's 160 KB.
static inline hipError_t check_lds(const void* kernel, size_t dynamic_bytes) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, kernel);
    if (e != hipSuccess) return e;
    return a.sharedSizeBytes + dynamic_bytes <= (size_t)VR_LDS_CU ? hipSuccess : hipErrorInvalidValue;
}

template <int MODE, int DT, int INTERP>
static hipError_t launch_r(const DevReq& R, const int* order, DevCounters* cnt, hipStream_t s) {
    const int grid = R.tiles_x * R.tiles_y;
    const size_t lds = (MODE == 0 ? (size_t)R.tf.n * 32 : (size_t)VR_MIPC_BYTES) + 2 * (size_t)R.box_bytes;
    const hipError_t e = check_lds((const void*)k_render<MODE, DT, INTERP>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_render<MODE, DT, INTERP>), dim3(grid), dim3(VR_WG), lds, s, R, order, cnt);
    return hipGetLastError();
}

// Persistent grid over the (request, tile) items of one batch class: items
// [hdr[2 + cls], hdr[3 + cls]) of the ordered work list, taken one at a time
// through the class's counter.  Which workgroup renders a tile never changes
// the tile's pixels.
template <int MODE, int DT, int INTERP>
__global__ __launch_bounds__(VR_WG, VR_WAVES_PER_EU) void k_render_batch(const DevReq* __restrict__ reqs,
                                                                         const DevItem* __restrict__ items,
                                                                         const int* __restrict__ hdr, int cls,
                                                                         unsigned* head, DevCounters* cnt) {
    extern __shared__ float4 lds4[];
    __shared__ int s_item;
    __shared__ unsigned wgc[5];
    __shared__ TileShared sh;
    float* tfl = (float*)lds4;
    const int i0 = hdr[2 + cls], i1 = hdr[3 + cls];
    for (;;) {
        if (threadIdx.x == 0) s_item = i0 + (int)atomicAdd(head, 1u);
        if (cnt && threadIdx.x < 5) wgc[threadIdx.x] = 0u;
        __syncthreads();
        const int it = s_item;
        if (it >= i1) break;
        const DevItem item = items[it];
        const DevReq& R = reqs[item.req];
        if (MODE == 0) tf_stage(R, lds4);
        const int tx = item.tile % R.tiles_x, ty = item.tile / R.tiles_x;
        LaneCounts c = {0u, 0u, 0u, 0u, 0u};
        uint8_t* boxes = (uint8_t*)tfl + (MODE == 0 ? 32 * R.tf.n : VR_MIPC_BYTES);
        render_tile_any<MODE, DT, INTERP>(R, tx, ty, tfl, boxes, sh, c);
        if (cnt) flush_counts(c, cnt + item.req, wgc);
        __syncthreads();
    }
}

template <int MODE, int DT, int INTERP>
static hipError_t launch_b(const DevReq* reqs, const DevItem* sorted, const int* hdr, int cls,
                           unsigned* head, DevCounters* cnt, size_t lds, int grid, hipStream_t s) {
    const hipError_t e = check_lds((const void*)k_render_batch<MODE, DT, INTERP>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_render_batch<MODE, DT, INTERP>), dim3(grid), dim3(VR_WG), lds, s, reqs, sorted,
                       hdr, cls, head + cls, cnt);
    return hipGetLastError();
}

// Defines the launchers of one (mode, storage) pair, both interpolations: the
// single image and the batch class.
#define VR_RENDER_LAUNCHER(MODE, DT)                                                          \
    hipError_t vr_launch_render_##MODE##_##DT(const DevReq& R, const int* order,               \
                                              DevCounters* cnt, hipStream_t s) {              \
        return R.interp == 1 ? launch_r<MODE, DT, 1>(R, order, cnt, s)                         \
                             : launch_r<MODE, DT, 0>(R, order, cnt, s);                        \
    }                                                                                          \
    hipError_t vr_launch_batch_##MODE##_##DT(const DevReq* reqs, const DevItem* sorted,        \
                                             const int* hdr, int interp, unsigned* head,       \
                                             DevCounters* cnt, size_t lds, int grid,           \
                                             hipStream_t s) {                                  \
        const int cls = VR_BATCH_CLASS(MODE, DT, interp);                                      \
        return interp == 1 ? launch_b<MODE, DT, 1>(reqs, sorted, hdr, cls, head, cnt, lds, grid, s) \
                           : launch_b<MODE, DT, 0>(reqs, sorted, hdr, cls, head, cnt, lds, grid, s); \
    }
