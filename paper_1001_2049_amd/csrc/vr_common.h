// vr_common.h — device-side storage formats shared by the HIP translation units.
#pragma once

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


