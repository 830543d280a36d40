// vr_host.h — host-side objects behind the C interface (context, cubes,
// transfer functions) and helpers shared by the API and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vr.h"
#include "vr_dev.h"

namespace vrh {

void set_error(const std::string& msg);

struct Ctx;

// Device memory owned by the library, allocated through the context's allocator.
struct DevBuf {
    void* ptr = nullptr;
    uint64_t bytes = 0;
};

// Work that reads an object, tracked with one event per stream that used it:
// the object may be freed or rewritten only once every stream's last use has
// completed (a single "last use" event would miss earlier readers on other
// streams).
struct Uses {
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
    vr_status record(hipStream_t s);        // after the work just enqueued on s
    vr_status wait_on(hipStream_t s) const; // make s wait for every recorded use
    vr_status sync() const;                 // the host waits for every recorded use
    bool done() const;                      // every recorded use has completed (no wait)
    bool has(hipStream_t s) const;          // a use on s has been recorded before
    void destroy();
};

struct MaskEntry {
    int mode = 0;
    int64_t tf_version = -1;
    uint32_t clip_bits = 0;
    DevBuf buf;                     // per slot 64-bit masks
    DevBuf bits;                    // per-cell grid
    DevBuf cellmax;                 // MIP: per-cell running-maximum bounds (grid order)
    hipEvent_t ready = nullptr;     // recorded after the classification that filled it
    Uses uses;                      // work reading it
    uint64_t stamp = 0;
};

struct Cube {
    vr_cube id = 0;
    int64_t nx = 0, ny = 0, nz = 0;
    int storage = VR_F32;
    double sigma = 1.0;
    int Bx = 0, By = 0, Bz = 0;
    int nslots = 0;
    int xch = 0;                    // x chunks per slot row
    uint64_t stride = 0;
    DevBuf pool, cellmm;
    std::deque<MaskEntry> masks;    // deque: entries never move while requests point at them
    Uses uses;                      // work reading this cube
    int refs = 0;                   // queued serving requests
    // Cubes registered with a host source are admitted to device memory on
    // demand and may be evicted while idle; uploaded cubes stay resident.
    const void* host_src = nullptr; // caller-owned voxels (registered cubes)
    int src_dtype = VR_F32;
    bool resident = false;
    // A registered cube larger than the budget is streamed: its statistics stay
    // on the device, its bricks in pinned host memory, and renders upload
    // groups of brick layers as sub-cubes (vr_render only).
    bool streamed = false;
    void* host_pool = nullptr;      // pinned: every slot, in slot order
    // Its two device buffers of sub-cubes stay allocated between frames (freed
    // with its device memory or when the budget needs room), each tagged with
    // the sub-cube it holds (-1: none) for sub-cubes of sbuf_G brick layers;
    // frames walk the sub-cubes in alternating order, so a frame starts on the
    // two sub-cubes the frame before ended with.
    DevBuf sbuf[2];
    int sbuf_sub[2] = {-1, -1};
    int sbuf_G = 0;
    bool sbuf_rev = false;
    int pins = 0;                   // served requests that have started on it
    uint64_t lru = 0;               // last admission or use, in ctx->lru_clock ticks
    // Coarse levels for the progressive loop (levels[L - 1]: 2x2x2 block means
    // of level L - 1, float32), built on demand within the budget and freed
    // with the cube's device memory or when the budget needs room.
    std::vector<std::unique_ptr<Cube>> levels;
    uint64_t bytes() const;
    uint64_t need_bytes() const;    // device bytes of its pool and statistics
};

struct Tf {
    vr_tf id = 0;
    int64_t version = 0;
    int n = 0;
    float v0 = 0.0f, v1 = 1.0f;
    std::vector<float> rows;  // n x 4
    DevBuf dev_rows;          // 2n float4: row, next row - row
    DevBuf dev_kpos;          // n + 2 ints: prefix counts of kappa > 0
    Uses uses;                // work reading this table
    bool internal = false;    // created by vr_set_transfer_function
    int refs = 0;             // queued serving requests
};

struct Server;

// Device and pinned staging for one persistent batched launch, and the
// graphs captured over those buffers (one per shape class).
struct BatchBufs {
    DevBuf reqs, items, head, hdr;
    DevBuf sorted;  // work list, each request's tiles most expensive first
    DevReq* pin_reqs = nullptr;
    DevItem* pin_items = nullptr;
    int* pin_hdr = nullptr;
    int reqs_cap = 0, items_cap = 0;
    hipEvent_t done = nullptr;  // staging is reusable once this has fired
    std::map<uint64_t, hipGraphExec_t> graphs;  // key: (items class, requests class, batch classes, LDS bytes)
};

struct Ctx {
    int device = -1;
    uint64_t budget = 0;
    uint64_t used = 0;
    bool has_alloc = false;
    vr_allocator alloc{};
    int num_cu = 256;
    std::recursive_mutex mu;

    // current state for vr_render
    bool has_camera = false;
    vr_camera camera{};
    vr_tf current_tf = 0;
    float clip = -__builtin_huge_valf();

    std::map<vr_cube, std::unique_ptr<Cube>> cubes;
    std::map<vr_tf, std::unique_ptr<Tf>> tfs;
    int32_t next_cube = 1, next_tf = 1;
    int64_t next_tf_version = 1;
    uint64_t mask_stamp = 0;
    uint64_t lru_clock = 0;
    uint64_t uploads = 0, evictions = 0;  // on-demand admissions of registered cubes
    uint64_t launch_stamp = 0;  // mask_stamp when the current launch began: newer entries are in use

    // scratch for single renders / batches
    DevBuf counters;             // DevCounters x capacity
    int counters_cap = 0;
    DevBuf order, ohist;         // single-render dispatch order and its bucket counts
    int order_cap = 0;
    hipEvent_t order_done = nullptr;  // last render that read `order`
    // Single renders compute each frame's dispatch order on a side stream into
    // one of two buffers (cap ints, then 256 histogram words), so that it can
    // run while the frame before is still rendering.
    DevBuf order2[2];
    int order2_cap = 0, order2_next = 0;
    bool order2_used[2] = {false, false};
    hipEvent_t order2_free[2] = {nullptr, nullptr};  // last render that read the buffer
    hipEvent_t order2_ready = nullptr;
    hipStream_t order_side = nullptr;
    BatchBufs batch;

    // progressive (coarse-to-fine) rendering: the view of the last call, the
    // level it delivered, and measured device time per nominal sample
    struct Progressive {
        bool valid = false;
        std::vector<uint8_t> key;   // cube, parameters, camera, transfer function, clip, output
        int level = 0;              // level delivered for this view
        double ms_per_sample = 0.0; // running estimate (0: none yet)
        uint64_t last_samples = 0;
        DevBuf low;                 // reduced-resolution image of a coarse level
        DevCounters* counters = nullptr;
        // transfer functions of coarse levels (extinction scaled by 2^L), by
        // (version of the table they derive from, L)
        std::map<std::pair<int64_t, int>, std::unique_ptr<Tf>> level_tfs;
    } prog;

    // The server is shared with callers blocked in vr_wait / vr_poll, so that a
    // concurrent vr_server_stop cannot free it under them.
    std::shared_ptr<Server> server;
    std::mutex server_mu;       // guards server start/stop

    bool host_only() const { return device < 0; }
};

// allocation through the context's allocator, counted against its budget
vr_status dev_alloc(Ctx* c, DevBuf& b, uint64_t bytes, bool budgeted);
void dev_free(Ctx* c, DevBuf& b, bool budgeted);

vr_status hip_check(hipError_t e, const char* what);

// validation helpers
vr_status check_camera(const vr_camera* cam);
vr_status check_params(const vr_render_params* p);
vr_status check_tf(const float* rgbk, int32_t n, float v0, float v1);

// camera constants for the kernels (float64 on the host, float-float to the device)
void camera_setup(const vr_camera& cam, int W, int H, DevCam& out);

// fill a DevReq for one image; classifies the skip mask on `s` if needed
// (prepared_only: never classify or allocate; VR_ESTATE if the mask is absent)
vr_status build_request(Ctx* c, Cube* cube, Tf* tf, float clip, const vr_camera& cam,
                        const vr_render_params& p, void* out, hipStream_t s, DevReq& R,
                        MaskEntry** mask_used, bool prepared_only = false);

// Allocation-free renders: per-device set-up at context creation.
vr_status noalloc_setup(int device);

// mark objects used by work enqueued on s
vr_status mark_use(Ctx* c, Cube* cube, Tf* tf, MaskEntry* mask, hipStream_t s);

Cube* find_cube(Ctx* c, vr_cube id);

// Make a cube's voxels resident on the device.  A registered cube that is not
// resident is uploaded from its host source after evicting idle registered
// cubes, least recently used first, until it fits the budget.  Cubes in
// `keep` (those of the launch being formed) are never evicted.  may_wait:
// wait for an idle candidate's queued work before evicting it; otherwise a
// candidate with work in flight is passed over.  Returns VR_EBUSY when the
// cube cannot be admitted now but might be once work completes, VR_ENOMEM
// when it cannot be admitted at all.
vr_status ensure_resident(Ctx* c, Cube* cube, hipStream_t s, bool may_wait,
                          const std::vector<Cube*>& keep);
Tf* find_tf(Ctx* c, vr_tf id);

// one persistent launch over many requests (used by vr_render_batch and the server);
// `tiles` optionally restricts request r to tiles [tiles[2r], tiles[2r+1]).  With
// use_graph the copies and kernels are replayed from a graph captured per
// shape class (stream s must not be the null stream).
vr_status launch_requests(Ctx* c, BatchBufs& bb, const vr_request* reqs, int count,
                          const int32_t* tiles, hipStream_t s, DevCounters* dev_counters,
                          bool use_graph = false);
void free_batch_bufs(Ctx* c, BatchBufs& bb);
vr_status check_request(Ctx* c, const vr_request* r);

}  // namespace vrh
