// vr_dev.h — plain structs passed from host to the HIP kernels, and the
// float-float ("double-single") arithmetic used for per-ray geometry.
//
// Ray set-up (camera ray, ray/box chord, sample-lattice anchors) runs in
// float-float arithmetic: a value is an unevaluated sum hi + lo of two floats,
// about 48 significant bits.  The error-free transformations are Knuth's
// TwoSum, Dekker's Fast2Sum and the FMA-based TwoProduct (Dekker 1971;
// Muller et al., Handbook of Floating-Point Arithmetic, ch. 4).  Per-sample
// work stays in plain float on coordinates local to a brick, so every sample
// position is accurate to a few 1e-6 voxel anywhere in a 2048^3 cube.
#pragma once

#include <stdint.h>

struct ff {
    float hi, lo;
};

// Layout and launch shape shared with the host.
#define VR_BRICK 32                 // brick edge (voxels)
#define VR_BRICK_APRON 33           // stored edge: brick plus one apron voxel
#define VR_CELL 8                   // skip-cell edge (voxels)
#define VR_CELLS_PER_BRICK 64       // 4 x 4 x 4
// Render workgroups: VR_WG threads own a VR_TW x VR_TH pixel tile, one 8x8
// block per wave, and VR_WG_PER_CU of them share a compute unit's LDS.
#ifndef VR_TW
#define VR_TW 16                    // workgroup tile width (pixels)
#endif
#ifndef VR_TH
#define VR_TH 16                    // workgroup tile height (pixels)
#endif
#define VR_WG (VR_TW * VR_TH)       // threads per render workgroup (one per pixel)
#define VR_NWAVE (VR_WG / 64)
#ifndef VR_WG_PER_CU
#define VR_WG_PER_CU 2              // render workgroups resident per compute unit
#endif
#define VR_LDS_CU 163840            // LDS per compute unit on gfx950
#define VR_LDS_MAX (VR_LDS_CU / VR_WG_PER_CU)  // LDS per render workgroup
#define VR_LDS_STATIC 4096          // reserved for the kernels' static LDS
// Slab boxes are sized against this many bytes (per buffer, two buffers),
// whatever LDS a launch actually leaves free, so that the image never depends
// on it; it fits beside a 256-row transfer function.
#ifndef VR_BOX_REF
#define VR_BOX_REF (VR_WG_PER_CU == 1 ? 73728 : (VR_LDS_MAX - VR_LDS_STATIC - 32 * 256) / 32 * 16)
#endif
// MIP running-maximum skipping keeps, per slab box, one bound per 8^3 cell in
// LDS (three slabs in flight) where the transfer function would otherwise sit.
#define VR_MIPC (768 / VR_WG_PER_CU)          // cells per slab box
#define VR_MIPC_BYTES (3 * VR_MIPC * 4)
#define VR_TROW 16                            // cells per box row (longer rows: no skipping)
// Batch class of a request: its kernel specialisation (mode, storage,
// interpolation); a batch runs one persistent launch per class present.
#define VR_NCLASS 12
#define VR_BATCH_CLASS(mode, dtype, interp) ((mode) * 6 + (dtype) * 2 + (interp))
#define VR_MAX_PARTIALS 64                    // sub-cube partials per composite
#define VR_PROG_LEVELS 5                      // progressive rendering: levels 0 .. 4
// Waves of the render kernels per SIMD (what the register budget must allow).
#define VR_WAVES_PER_EU ((VR_NWAVE * VR_WG_PER_CU + 3) / 4)
// Brick slot layout.  A slot stores local voxels x in [0, 4*xch), y in [0, 36),
// z in [0, 34) (the brick's 33^3 with its apron, padded), each the
// edge-clamped value of its global position.  Memory is cut into 128-byte
// lines; a line holds one 16-byte chunk of x (4 float or 8 16-bit values) for
// 4 consecutive y and 2 consecutive z, so that a box of any orientation copied
// chunk by chunk uses whole lines.  The element offset of (lx, ly, lz) is
// X(lx) + Y(ly) + Z(lz) with
//   X = (lx / CV) * 8 CV + lx % CV,  Y = (ly / 4) * xch * 8 CV + (ly % 4) * CV,
//   Z = (lz / 2) * 9 * xch * 8 CV + (lz % 2) * 4 CV.
#define VR_SLOT_YG 9                // groups of 4 rows per slot
#define VR_SLOT_ZP 17               // pairs of planes per slot
#define VR_XCH(dt) ((dt) == 0 ? 9 : 5)   // x chunks per row
#define VR_CVE(dt) ((dt) == 0 ? 4 : 8)   // elements per 16-byte chunk

// Cube as seen by the render kernels.  Slot of brick (bx, by, bz) is the
// linear index (bz * by_count + by) * bx_count + bx.
struct DevCube {
    const uint8_t* pool;            // brick slots
    const uint64_t* mask;           // per slot: bit c set if cell c may contribute
    const uint32_t* cellbits;       // per cell (x fastest, 4 cells per brick edge): may contribute
    const float* cellmax;           // MIP, per cell in the same order: a bound on every value its
                                    // samples can take if the cell can reach the clip, else -inf
                                    // (NULL: no running-maximum skipping)
    uint64_t stride;                // bytes per slot
    int32_t nx, ny, nz;
    int32_t bx, by, bz;             // bricks per axis
    int32_t dtype;                  // 0 f32, 1 f16, 2 bf16
    int32_t xch;                    // x chunks per slot row
    int32_t bz_hi;                  // brick layers below this one are addressable (bz normally;
                                    // a streamed sub-cube holds only some layers, and planes
                                    // above them are read from the top layer's apron)
};

// Transfer function: rows[2i] = row i (r, g, b, kappa), rows[2i+1] = row i+1 - row i.
struct DevTf {
    const float* rows;              // 8 floats per row
    int32_t n;
    float scale, bias;              // u = stored_value * scale + bias
    float clip;                     // in stored units; -inf: none
};

// Camera constants in float-float.  Perspective: origin o, direction of pixel
// (i, j) before normalisation base + (i+1/2) dx + (j+1/2) dy.  Orthographic:
// origin o + (i+1/2) dx + (j+1/2) dy, direction dir.
struct DevCam {
    ff o[3], base[3], dx[3], dy[3], dir[3];
    int32_t ortho;
    int32_t pad;
};

// One render request (a whole image).
struct DevReq {
    DevCube cube;
    DevTf tf;
    DevCam cam;
    float* out;                     // [H][W][4] (EA) or [H][W] (MIP)
    int32_t W, H, tiles_x, tiles_y;
    int32_t mode, interp, use_skip;
    int32_t box_bytes;              // LDS bytes of one slab box buffer (two are used)
    ff step;                        // lattice spacing
    float ert_T;                    // stop once transmittance <= ert_T
    float out_scale;                // MIP: stored units -> data units
    // Sub-cube partial: only lattice samples whose position on axis win_axis
    // lies in [win_lo, win_hi) (the lattice stays the whole cube's); voxels
    // outside planes [win_vlo, win_vhi] on that axis are never read.
    int32_t win_axis;               // -1: whole rays
    int32_t win_vlo, win_vhi;
    int32_t partial;                // MIP partial encoding (see store_pixel)
    float win_lo, win_hi;
};

// Device counters (optional).
struct DevCounters {
    unsigned long long samples_nominal, samples_exec, rays_hit, rays_ert, cells_skipped, pad[3];
};

// One unit of batched work: one workgroup tile of a request.
struct DevItem {
    int32_t req, tile;
};

#if defined(__HIPCC__) || defined(__HIP_DEVICE_COMPILE__)
#define VR_FF_FN __device__ __forceinline__

VR_FF_FN ff ff_make(float hi) { return ff{hi, 0.0f}; }

VR_FF_FN ff two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return ff{s, e};
}

VR_FF_FN ff fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float e = b - (s - a);
    return ff{s, e};
}

VR_FF_FN ff two_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return ff{p, e};
}

VR_FF_FN ff ff_add(ff a, ff b) {
#pragma clang fp contract(off)
    ff s = two_sum(a.hi, b.hi);
    ff t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

VR_FF_FN ff ff_neg(ff a) { return ff{-a.hi, -a.lo}; }
VR_FF_FN ff ff_sub(ff a, ff b) { return ff_add(a, ff_neg(b)); }

VR_FF_FN ff ff_mul(ff a, ff b) {
#pragma clang fp contract(off)
    ff p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fmaf(a.hi, b.lo, __builtin_fmaf(a.lo, b.hi, p.lo));
    return fast_two_sum(p.hi, p.lo);
}

VR_FF_FN ff ff_mul_f(ff a, float b) {
#pragma clang fp contract(off)
    ff p = two_prod(a.hi, b);
    p.lo = __builtin_fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

VR_FF_FN ff ff_div(ff a, ff b) {
#pragma clang fp contract(off)
    float q1 = a.hi / b.hi;
    ff r = ff_sub(a, ff_mul_f(b, q1));
    float q2 = r.hi / b.hi;
    r = ff_sub(r, ff_mul_f(b, q2));
    float q3 = r.hi / b.hi;
    ff q = fast_two_sum(q1, q2);
    return ff_add(q, ff{q3, 0.0f});
}

VR_FF_FN ff ff_sqrt(ff a) {
#pragma clang fp contract(off)
    if (!(a.hi > 0.0f)) return ff{0.0f, 0.0f};
    float s = __builtin_sqrtf(a.hi);
    ff s2 = two_prod(s, s);
    float r = ((a.hi - s2.hi) - s2.lo + a.lo) / (2.0f * s);
    return fast_two_sum(s, r);
}

VR_FF_FN bool ff_lt(ff a, ff b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
// field-wise selects: a select of whole structs would go through stack memory
VR_FF_FN ff ff_sel(bool c, ff a, ff b) {
    ff r;
    r.hi = c ? a.hi : b.hi;
    r.lo = c ? a.lo : b.lo;
    return r;
}
VR_FF_FN ff ff_min(ff a, ff b) { return ff_sel(ff_lt(b, a), b, a); }
VR_FF_FN ff ff_max(ff a, ff b) { return ff_sel(ff_lt(a, b), b, a); }
VR_FF_FN float ff_to_f(ff a) { return a.hi + a.lo; }
#endif
