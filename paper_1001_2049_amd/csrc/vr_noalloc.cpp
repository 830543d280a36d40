// vr_noalloc.cpp — vr_render_noalloc: one render that allocates nothing.
//
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid it).  vr_render draws its
// dispatch-order scratch (per-tile order and bucket counts) from buffers the
// context allocates on demand; this entry point takes it from a fixed array
// in device memory instead, `scratch` below.  Every GPU the library runs on
// holds its own copy of the array until the process ends.  Its address on a
// device is looked up once, when a context is created on that device (host
// code must never pass the array's name itself: that is a host-side stand-in
// for the symbol, not a device address).
//
// All calls on one GPU share that GPU's array: calls that overlap on one GPU
// (on different streams, or from different contexts) race on it.  The bucket
// counts are cleared by a kernel at the start of every call.
#include <cstring>
#include <map>
#include <mutex>

#include "vr_host.h"
#include "vr_launch.h"

#define VR_NOALLOC_TILES 262144        // 16x16-pixel tiles: e.g. 8192 x 8192 pixels
#define VR_NOALLOC_ORDER_BYTES (VR_NOALLOC_TILES * 4)
#define VR_NOALLOC_BYTES (VR_NOALLOC_ORDER_BYTES + 1024)

static __device__ __align__(256) unsigned char scratch[VR_NOALLOC_BYTES];

namespace vrh {

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device -> device address of `scratch`

vr_status noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return VR_OK;
    void* ptr = nullptr;
    vr_status st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st == VR_OK) st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (st != VR_OK) return st;
    g_scratch_ptr[device] = ptr;
    return VR_OK;
}

static void* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

}  // namespace vrh

using namespace vrh;

extern "C" vr_status vr_render_noalloc(vr_ctx ctx, vr_cube cube, const vr_render_params* params,
                                       void* out_dev, void* hip_stream) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    vr_status st = check_params(params);
    if (st != VR_OK) return st;
    if (!out_dev) {
        set_error("out_dev is NULL");
        return VR_EINVAL;
    }
    const int64_t tiles = (int64_t)((params->width + VR_TW - 1) / VR_TW) *
                          ((params->height + VR_TH - 1) / VR_TH);
    if (tiles > VR_NOALLOC_TILES) {
        set_error("image of " + std::to_string(tiles) + " tiles exceeds the fixed scratch of " +
                  std::to_string(VR_NOALLOC_TILES) + " tiles");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    try {
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot render");
            return VR_EDEVICE;
        }
        if (!c->has_camera) {
            set_error("camera not set");
            return VR_ESTATE;
        }
        Tf* tf = nullptr;
        if (params->mode == VR_EA) {
            if (!c->current_tf) {
                set_error("transfer function not set");
                return VR_ESTATE;
            }
            tf = find_tf(c, c->current_tf);
        }
        Cube* cu = find_cube(c, cube);
        if (!cu) {
            set_error("unknown cube handle " + std::to_string(cube));
            return VR_ENOTFOUND;
        }
        hipStream_t s = (hipStream_t)hip_stream;
        // nothing may be allocated: the cube must be resident and every object
        // the render reads must have a use already tracked on this stream
        if (!cu->resident || !cu->uses.has(s) || (tf && !tf->uses.has(s))) {
            set_error("cube or transfer function not prepared on this stream (render it once with "
                      "vr_render on this stream first)");
            return VR_ESTATE;
        }
        st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        uint8_t* base = (uint8_t*)scratch_of(c->device);
        if (!base) {
            set_error("scratch of this device was not set up");
            return VR_EDEVICE;
        }
        DevReq R;
        MaskEntry* me = nullptr;
        st = build_request(c, cu, tf, c->clip, c->camera, *params, out_dev, s, R, &me, true);
        if (st != VR_OK) return st;
        if (me && !me->uses.has(s)) {
            set_error("skip mask not prepared on this stream (render it once with vr_render on "
                      "this stream first)");
            return VR_ESTATE;
        }
        st = hip_check(vr_launch_render(R, (int*)base, (unsigned*)(base + VR_NOALLOC_ORDER_BYTES),
                                        nullptr, s),
                       "render launch");
        if (st != VR_OK) return st;
        return mark_use(c, cu, tf, me, s);
    } catch (...) {
        set_error("internal error");
        return VR_EINVAL;
    }
}
