// synth_gpu.hip — the synthetic cube generator of synth.c, evaluated on the GPU.
//
// Input generator only (no rendering arithmetic).  It produces, voxel by voxel,
// the same sum as synth_cube(): sigma * N(0,1) from Philox4x32-10 and the
// Box-Muller transform in double precision, plus the Gaussian sources in
// catalogue order, rounded once to float.  Everything that depends on the
// sources alone (the per-plane factor A * sigma * G_z and the per-source x and
// y factors) is evaluated by the caller on the CPU with the C library's exp
// and passed in as tables, so the source terms are bit-identical to the CPU
// generator's; the noise uses the device's double-precision log, sqrt, sin and
// cos, which can differ from the C library's in the last bit, so a voxel can
// (rarely) differ from the CPU value by one float rounding step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#pragma clang fp contract(off)

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

__device__ static double normal_dev(uint64_t seed, uint64_t v) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);  // noise stream 0
    const uint64_t pair = v >> 1;
    uint32_t c0 = (uint32_t)pair, c1 = (uint32_t)(pair >> 32), c2 = 0, c3 = 0;
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    const double u1 = 1.0 - ((double)(c0 >> 5) * 67108864.0 + (double)(c1 >> 6)) * (1.0 / 9007199254740992.0);
    const double u2 = ((double)(c2 >> 5) * 67108864.0 + (double)(c3 >> 6)) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586476925286766559 * u2;
    return (v & 1) ? r * sin(ang) : r * cos(ang);
}

// Planes z0 .. z0+nzs-1.  Entry k of plane zz (plane_off[zz] <= k < plane_off[zz+1],
// in catalogue order) is source ent_src[k] with factor ent_a[k] = A sigma G_z;
// source s covers x in [rect[4s], rect[4s+1]] and y in [rect[4s+2], rect[4s+3]]
// with factors fx[fx_off[s] + x - x_a] and fy[fy_off[s] + y - y_a].
__global__ void k_synth(uint64_t seed, int64_t nx, int64_t ny, double sigma, int noise, int64_t z0,
                        int64_t nzs, const int64_t* plane_off, const int32_t* ent_src,
                        const double* ent_a, const int32_t* rect, const int64_t* fx_off,
                        const int64_t* fy_off, const double* fx, const double* fy, float* out) {
    const int64_t per_plane = nx * ny;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per_plane * nzs) return;
    const int64_t zz = i / per_plane, rem = i - zz * per_plane;
    const int32_t y = (int32_t)(rem / nx), x = (int32_t)(rem - (int64_t)y * nx);
    double acc = noise ? sigma * normal_dev(seed, (uint64_t)(z0 + zz) * (uint64_t)per_plane + (uint64_t)rem)
                       : 0.0;
    for (int64_t k = plane_off[zz]; k < plane_off[zz + 1]; ++k) {
        const int32_t s = ent_src[k];
        const int32_t xa = rect[4 * s], xb = rect[4 * s + 1], ya = rect[4 * s + 2], yb = rect[4 * s + 3];
        if (x < xa || x > xb || y < ya || y > yb) continue;
        const double ay = ent_a[k] * fy[fy_off[s] + (y - ya)];
        acc += ay * fx[fx_off[s] + (x - xa)];
    }
    out[i] = (float)acc;
}

extern "C" int synth_gpu_planes(uint64_t seed, int64_t nx, int64_t ny, double sigma, int noise,
                                int64_t z0, int64_t nzs, const int64_t* plane_off,
                                const int32_t* ent_src, const double* ent_a, const int32_t* rect,
                                const int64_t* fx_off, const int64_t* fy_off, const double* fx,
                                const double* fy, float* out_dev, int device, void* stream) {
    const int64_t total = nx * ny * nzs;
    if (total <= 0) return 0;
    hipError_t se = hipSetDevice(device);
    if (se != hipSuccess) return -2000 - (int)se;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return -1;
    (void)hipGetLastError();  // an error left by earlier, unrelated calls is not ours
    hipLaunchKernelGGL(k_synth, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, seed, nx, ny,
                       sigma, noise, z0, nzs, plane_off, ent_src, ent_a, rect, fx_off, fy_off, fx, fy,
                       out_dev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : -1000 - (int)e;
}
