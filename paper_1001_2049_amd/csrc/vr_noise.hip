// vr_noise.hip — per-channel noise estimation for the noise-aware form.
//
// A spectral cube's noise level varies with frequency; the paper singles out
// data of low signal-to-noise ratio (abstract; Sec. 2).  Each frequency
// channel (z plane) gets a robust noise estimate: the lower median of its
// values, the lower median of the absolute deviations from it (MAD, taken on
// float32 deviations: rounding is monotone, so this is the exact MAD rounded
// once), and sigma = 1.4826 MAD.  Both medians are exact order statistics found
// by a most-significant-digit radix selection over the float keys: one
// workgroup per channel, four passes of 8 bits, a 256-bin LDS histogram per
// pass, each pass narrowing the key prefix to the bin holding the wanted rank.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr_common.h"
#include "vr_launch.h"

#define VR_SEL_WG 512

// order-preserving map of float to unsigned (total order of non-NaN floats)
__device__ __forceinline__ uint32_t float_key(float v) {
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __builtin_bit_cast(float, u);
}

// Key of rank `rank` (0-based) among the n keys produced by key_of(i).
template <typename KeyOf>
__device__ uint32_t select_rank(KeyOf key_of, int64_t n, int64_t rank, unsigned* hist,
                                uint32_t* shared_word) {
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += VR_SEL_WG) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += VR_SEL_WG) {
            const uint32_t k = key_of(i);
            if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // the bin holding the wanted rank (256 bins, one thread: negligible)
            int64_t below = 0;
            int b = 0;
            for (; b < 255; ++b) {
                if (below + (int64_t)hist[b] > rank) break;
                below += hist[b];
            }
            shared_word[0] = (uint32_t)b;
            shared_word[1] = (uint32_t)below;
        }
        __syncthreads();
        const uint32_t b = shared_word[0];
        rank -= (int64_t)shared_word[1];
        prefix |= b << shift;
        mask |= 255u << shift;
        __syncthreads();
    }
    return prefix;
}

// One workgroup per channel z of `planes` consecutive channels starting at
// plane z_first of the cube (src holds those planes, x fastest).
__global__ __launch_bounds__(VR_SEL_WG) void k_channel_noise(const float* __restrict__ src,
                                                             int64_t plane, int64_t z_first,
                                                             float* __restrict__ med_out,
                                                             float* __restrict__ mad_out,
                                                             float* __restrict__ sigma_out) {
    __shared__ unsigned hist[256];
    __shared__ uint32_t word[2];
    const float* p = src + (int64_t)blockIdx.x * plane;
    const int64_t rank = (plane - 1) / 2;
    const float med = key_float(select_rank([&](int64_t i) { return float_key(p[i]); }, plane, rank,
                                            hist, word));
    const float mad = key_float(select_rank(
        [&](int64_t i) { return float_key(fabsf(p[i] - med)); }, plane, rank, hist, word));
    if (threadIdx.x == 0) {
        const int64_t z = z_first + blockIdx.x;
        med_out[z] = med;
        mad_out[z] = mad;
        sigma_out[z] = (float)(1.4826 * (double)mad);
    }
}

hipError_t vr_launch_channel_noise(const float* src, int64_t plane, int64_t z_first, int planes,
                                   float* med, float* mad, float* sigma, hipStream_t s) {
    if (planes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_channel_noise, dim3(planes), dim3(VR_SEL_WG), 0, s, src, plane, z_first,
                       med, mad, sigma);
    return hipGetLastError();
}
