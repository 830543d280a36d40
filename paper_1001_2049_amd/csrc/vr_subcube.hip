// vr_subcube.hip — scene integration of sub-cube partial images.
//
// The paper splits the cube into sub-cubes, renders each to an image and
// combines the images in a final step (Sec. 3.1, process steps 1, 4 and 5).
// A partial here is rendered on the lattice of the whole cube (vr_render_subcube),
// so the partials of a split compose into the image of the whole cube:
// emission-absorption partials (premultiplied RGBA) by front-to-back "over"
// (Porter and Duff 1984) in the order each pixel's ray crosses them, and MIP
// partials by their maximum, floored at the clip.
#include "vr_render.h"

struct PartialList {
    const float* p[VR_MAX_PARTIALS];
};

__global__ __launch_bounds__(256) void k_composite(const PartialList L, int count, int mode,
                                                   int axis, const DevCam cam, int W, int H,
                                                   float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    if (mode == 1) {
        float m = -VR_INF;
        for (int k = 0; k < count; ++k) m = fmaxf(m, L.p[k][i]);
        out[i] = m == -3.402823466e38f ? 0.0f : m;  // samples, all below the clip
        return;
    }
    const int x = (int)(i % W), y = (int)(i / W);
    ff o[3], d[3];
    ray_dir(cam, (float)x + 0.5f, (float)y + 0.5f, o, d);
    const float da = axis == 0 ? d[0].hi : (axis == 1 ? d[1].hi : d[2].hi);
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int q = 0; q < count; ++q) {
        const int k = da >= 0.0f ? q : count - 1 - q;
        const float4 c = ((const float4*)L.p[k])[i];
        const float t = 1.0f - acc.w;
        acc.x = __builtin_fmaf(t, c.x, acc.x);
        acc.y = __builtin_fmaf(t, c.y, acc.y);
        acc.z = __builtin_fmaf(t, c.z, acc.z);
        acc.w = __builtin_fmaf(t, c.w, acc.w);
    }
    ((float4*)out)[i] = acc;
}

hipError_t vr_launch_composite(const float* const* partials, int count, int mode, int axis,
                               const DevCam& cam, int W, int H, float* out, hipStream_t s) {
    PartialList L;
    for (int k = 0; k < VR_MAX_PARTIALS; ++k) L.p[k] = k < count ? partials[k] : nullptr;
    const int64_t n = (int64_t)W * H;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, count,
                       mode, axis, cam, W, H, out);
    return hipGetLastError();
}
