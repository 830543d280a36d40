// vr_capi.cpp — the C interface: context, validation, cube upload (bricking),
// transfer functions, skip classification cache, single and batched renders.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "vr_host.h"
#include "vr_launch.h"
#include "vr_server.h"

namespace vrh {

static thread_local std::string g_err;
// step in progress, named in the message of an unexpected exception
static thread_local const char* g_stage = "";

void set_error(const std::string& msg) { g_err = msg; }

vr_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return VR_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return VR_EDEVICE;
}

vr_status Uses::record(hipStream_t s) {
    for (auto& e : ev)
        if (e.first == s) return hip_check(hipEventRecord(e.second, s), "hipEventRecord");
    if (ev.size() >= 16) {
        // bound the list: once every older use is complete, it can be dropped
        vr_status st = sync();
        if (st != VR_OK) return st;
        destroy();
    }
    hipEvent_t e = nullptr;
    vr_status st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    if (st != VR_OK) return st;
    ev.emplace_back(s, e);
    return hip_check(hipEventRecord(e, s), "hipEventRecord");
}

vr_status Uses::wait_on(hipStream_t s) const {
    for (const auto& e : ev) {
        if (e.first == s) continue;  // stream order already covers it
        vr_status st = hip_check(hipStreamWaitEvent(s, e.second, 0), "hipStreamWaitEvent");
        if (st != VR_OK) return st;
    }
    return VR_OK;
}

vr_status Uses::sync() const {
    for (const auto& e : ev) {
        vr_status st = hip_check(hipEventSynchronize(e.second), "hipEventSynchronize");
        if (st != VR_OK) return st;
    }
    return VR_OK;
}

bool Uses::has(hipStream_t s) const {
    for (const auto& e : ev)
        if (e.first == s) return true;
    return false;
}

bool Uses::done() const {
    for (const auto& e : ev) {
        const hipError_t q = hipEventQuery(e.second);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) (void)hipGetLastError();  // reported by the next synchronising call
    }
    return true;
}

void Uses::destroy() {
    for (auto& e : ev) (void)hipEventDestroy(e.second);
    ev.clear();
}

uint64_t Cube::bytes() const {
    uint64_t b = pool.bytes + cellmm.bytes;
    for (const auto& m : masks) b += m.buf.bytes + m.bits.bytes;
    return b;
}

static uint64_t alloc_size(uint64_t bytes) { return ((bytes ? bytes : 256) + 255) & ~uint64_t(255); }

uint64_t Cube::need_bytes() const {
    return alloc_size((uint64_t)nslots * stride) + alloc_size((uint64_t)nslots * 2 * VR_CELLS_PER_BRICK * 4);
}

vr_status dev_alloc(Ctx* c, DevBuf& b, uint64_t bytes, bool budgeted) {
    bytes = alloc_size(bytes);
    if (budgeted && c->budget && c->used + bytes > c->budget) {
        set_error("device memory budget exceeded (" + std::to_string(c->used + bytes) + " > " +
                  std::to_string(c->budget) + " bytes)");
        return VR_ENOMEM;
    }
    void* p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
        if (!p) {
            set_error("allocator returned NULL for " + std::to_string(bytes) + " bytes");
            return VR_ENOMEM;
        }
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            return VR_ENOMEM;
        }
    }
    b.ptr = p;
    b.bytes = bytes;
    if (budgeted) c->used += bytes;
    return VR_OK;
}

void dev_free(Ctx* c, DevBuf& b, bool budgeted) {
    if (!b.ptr) return;
    if (c->has_alloc) c->alloc.free(b.ptr, b.bytes, c->alloc.user);
    else (void)hipFree(b.ptr);
    if (budgeted) c->used -= b.bytes;
    b = DevBuf{};
}

static bool finite3(const double* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

vr_status check_camera(const vr_camera* cam) {
    if (!cam) {
        set_error("camera is NULL");
        return VR_EINVAL;
    }
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up)) {
        set_error("camera vectors must be finite");
        return VR_EINVAL;
    }
    double f[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1],
                   cam->target[2] - cam->eye[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    double ul = std::sqrt(cam->up[0] * cam->up[0] + cam->up[1] * cam->up[1] +
                          cam->up[2] * cam->up[2]);
    if (!(fl > 0.0) || !(ul > 0.0)) {
        set_error("camera: eye == target or zero up vector");
        return VR_EINVAL;
    }
    double r[3] = {f[1] * cam->up[2] - f[2] * cam->up[1], f[2] * cam->up[0] - f[0] * cam->up[2],
                   f[0] * cam->up[1] - f[1] * cam->up[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 1e-9 * fl * ul)) {
        set_error("camera: up is parallel to the view direction");
        return VR_EINVAL;
    }
    if (cam->ortho != 0 && cam->ortho != 1) {
        set_error("camera: ortho must be 0 or 1");
        return VR_EINVAL;
    }
    if (cam->ortho) {
        if (!(cam->ortho_w > 0.0) || !(cam->ortho_h > 0.0) || !std::isfinite(cam->ortho_w) ||
            !std::isfinite(cam->ortho_h)) {
            set_error("camera: orthographic window must be positive and finite");
            return VR_EINVAL;
        }
    } else if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) {
        set_error("camera: fovy_deg must lie in (0, 180)");
        return VR_EINVAL;
    }
    return VR_OK;
}

vr_status check_params(const vr_render_params* p) {
    if (!p) {
        set_error("render params are NULL");
        return VR_EINVAL;
    }
    if (p->mode != VR_EA && p->mode != VR_MIP) {
        set_error("mode must be VR_EA or VR_MIP");
        return VR_EINVAL;
    }
    if (p->interp != VR_NEAREST && p->interp != VR_TRILINEAR) {
        set_error("interp must be VR_NEAREST or VR_TRILINEAR");
        return VR_EINVAL;
    }
    if (!(p->step >= 1e-3f && p->step <= 1e6f)) {
        set_error("step must lie in [1e-3, 1e6] voxels");
        return VR_EINVAL;
    }
    if (!(p->ert_alpha > 0.0f) || std::isnan(p->ert_alpha)) {
        set_error("ert_alpha must be > 0 (values > 1 disable early termination)");
        return VR_EINVAL;
    }
    if (p->width < 1 || p->height < 1 || p->width > 16384 || p->height > 16384) {
        set_error("width and height must lie in [1, 16384]");
        return VR_EINVAL;
    }
    if (p->use_skip != 0 && p->use_skip != 1) {
        set_error("use_skip must be 0 or 1");
        return VR_EINVAL;
    }
    return VR_OK;
}

vr_status check_tf(const float* rgbk, int32_t n, float v0, float v1) {
    if (!rgbk) {
        set_error("transfer function table is NULL");
        return VR_EINVAL;
    }
    if (n < 2 || n > 4096) {
        set_error("transfer function needs 2..4096 rows");
        return VR_EINVAL;
    }
    if (!std::isfinite(v0) || !std::isfinite(v1) || !(v1 > v0)) {
        set_error("transfer function domain needs finite v0 < v1");
        return VR_EINVAL;
    }
    for (int i = 0; i < 4 * n; ++i) {
        if (!std::isfinite(rgbk[i])) {
            set_error("transfer function entries must be finite");
            return VR_EINVAL;
        }
        if (i % 4 == 3 && rgbk[i] < 0.0f) {
            set_error("extinction (4th channel) must be >= 0");
            return VR_EINVAL;
        }
    }
    return VR_OK;
}

static ff to_ff(double x) {
    ff v;
    v.hi = (float)x;
    v.lo = std::isfinite(x) ? (float)(x - (double)v.hi) : 0.0f;
    return v;
}

void camera_setup(const vr_camera& cam, int W, int H, DevCam& out) {
    double f[3], r[3], u[3];
    for (int a = 0; a < 3; ++a) f[a] = cam.target[a] - cam.eye[a];
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int a = 0; a < 3; ++a) f[a] /= fl;
    r[0] = f[1] * cam.up[2] - f[2] * cam.up[1];
    r[1] = f[2] * cam.up[0] - f[0] * cam.up[2];
    r[2] = f[0] * cam.up[1] - f[1] * cam.up[0];
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int a = 0; a < 3; ++a) r[a] /= rl;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    std::memset(&out, 0, sizeof(out));
    out.ortho = cam.ortho;
    if (cam.ortho) {
        const double w = cam.ortho_w, h = cam.ortho_h;
        for (int a = 0; a < 3; ++a) {
            out.o[a] = to_ff(cam.target[a] - 0.5 * w * r[a] + 0.5 * h * u[a]);
            out.dx[a] = to_ff((w / W) * r[a]);
            out.dy[a] = to_ff(-(h / H) * u[a]);
            out.dir[a] = to_ff(f[a]);
        }
    } else {
        const double h = std::tan(0.5 * cam.fovy_deg * (3.14159265358979323846 / 180.0));
        const double asp = (double)W / (double)H;
        for (int a = 0; a < 3; ++a) {
            out.o[a] = to_ff(cam.eye[a]);
            out.base[a] = to_ff(f[a] - h * asp * r[a] + h * u[a]);
            out.dx[a] = to_ff((2.0 * h * asp / W) * r[a]);
            out.dy[a] = to_ff(-(2.0 * h / H) * u[a]);
        }
    }
}

Cube* find_cube(Ctx* c, vr_cube id) {
    auto it = c->cubes.find(id);
    return it == c->cubes.end() ? nullptr : it->second.get();
}

Tf* find_tf(Ctx* c, vr_tf id) {
    auto it = c->tfs.find(id);
    return it == c->tfs.end() ? nullptr : it->second.get();
}

static vr_status ensure_event(hipEvent_t& e) {
    if (e) return VR_OK;
    return hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
}

// skip mask for (mode, transfer function, clip) on this cube, classified on s if absent
static vr_status get_mask(Ctx* c, Cube* cube, int mode, Tf* tf, float clip_s, hipStream_t s,
                          MaskEntry** out, bool may_create = true) {
    const int64_t ver = mode == VR_EA ? tf->version : -1;
    uint32_t cb;
    std::memcpy(&cb, &clip_s, 4);
    for (auto& m : cube->masks) {
        if (m.mode == mode && m.tf_version == ver && m.clip_bits == cb) {
            // the classification that filled it may have been enqueued on another stream
            vr_status st = hip_check(hipStreamWaitEvent(s, m.ready, 0), "hipStreamWaitEvent");
            if (st != VR_OK) return st;
            m.stamp = ++c->mask_stamp;
            *out = &m;
            return VR_OK;
        }
    }
    if (!may_create) {
        set_error("the skip mask of this cube, mode, transfer function and clip is not prepared "
                  "(render it once with vr_render on this stream)");
        return VR_ESTATE;
    }
    MaskEntry* e = nullptr;
    // evict the least recently used entry that the launch being built does not use
    MaskEntry* lru = nullptr;
    for (auto& m : cube->masks)
        if (m.stamp <= c->launch_stamp && (!lru || m.stamp < lru->stamp)) lru = &m;
    if (cube->masks.size() < 8 || !lru) {
        cube->masks.emplace_back();
        e = &cube->masks.back();
        // skip masks (about 0.01 % of a pool) are not counted against the budget
        vr_status st = dev_alloc(c, e->buf, (uint64_t)cube->nslots * 8, false);
        if (st == VR_OK)
            st = dev_alloc(c, e->bits, (uint64_t)vr_cellbits_words(cube->Bx, cube->By, cube->Bz) * 4,
                           false);
        if (st != VR_OK) {
            dev_free(c, e->buf, false);
            cube->masks.pop_back();
            return st;
        }
        st = ensure_event(e->ready);
        if (st != VR_OK) return st;
    } else {
        e = lru;
        // the entry may still be read by queued work on any stream that used it
        vr_status st = e->uses.wait_on(s);
        if (st != VR_OK) return st;
    }
    float scale = 1.0f, bias = 0.0f;
    int n = 2;
    const int* kpos = nullptr;
    if (mode == VR_EA) {
        const double k = (double)(tf->n - 1) / ((double)tf->v1 - (double)tf->v0);
        scale = (float)(cube->sigma * k);
        bias = (float)(-(double)tf->v0 * k);
        n = tf->n;
        kpos = (const int*)tf->dev_kpos.ptr;
    }
    if (mode == VR_MIP && !e->cellmax.ptr) {
        vr_status st = dev_alloc(c, e->cellmax, (uint64_t)cube->nslots * VR_CELLS_PER_BRICK * 4, false);
        if (st != VR_OK) return st;
    }
    vr_status st = hip_check(
        vr_launch_classify((const float*)cube->cellmm.ptr, (uint64_t*)e->buf.ptr,
                           (uint32_t*)e->bits.ptr, (float*)e->cellmax.ptr, cube->Bx, cube->By,
                           cube->Bz, mode, clip_s, scale, bias, n, kpos, s),
        "classify launch");
    if (st == VR_OK) st = hip_check(hipEventRecord(e->ready, s), "hipEventRecord");
    if (st != VR_OK) return st;
    e->mode = mode;
    e->tf_version = ver;
    e->clip_bits = cb;
    e->stamp = ++c->mask_stamp;
    *out = e;
    return VR_OK;
}

vr_status build_request(Ctx* c, Cube* cube, Tf* tf, float clip, const vr_camera& cam,
                        const vr_render_params& p, void* out, hipStream_t s, DevReq& R,
                        MaskEntry** mask_used, bool prepared_only) {
    std::memset(&R, 0, sizeof(R));
    R.win_axis = -1;
    if (mask_used) *mask_used = nullptr;
    // sample count per ray must stay exactly representable
    const double diag = std::sqrt((double)cube->nx * cube->nx + (double)cube->ny * cube->ny +
                                  (double)cube->nz * cube->nz);
    if (diag / p.step > 4.0e6) {
        set_error("step too small for this cube (more than 4e6 samples per ray)");
        return VR_EINVAL;
    }
    R.cube.pool = (const uint8_t*)cube->pool.ptr;
    R.cube.stride = cube->stride;
    R.cube.xch = cube->xch;
    R.cube.nx = (int)cube->nx;
    R.cube.ny = (int)cube->ny;
    R.cube.nz = (int)cube->nz;
    R.cube.bx = cube->Bx;
    R.cube.by = cube->By;
    R.cube.bz = cube->Bz;
    R.cube.dtype = cube->storage;
    R.cube.bz_hi = cube->Bz;
    const float clip_s = std::isfinite(clip) ? (float)((double)clip / cube->sigma) : clip;
    R.tf.clip = clip_s;
    if (p.mode == VR_EA) {
        const double k = (double)(tf->n - 1) / ((double)tf->v1 - (double)tf->v0);
        R.tf.rows = (const float*)tf->dev_rows.ptr;
        R.tf.n = tf->n;
        R.tf.scale = (float)(cube->sigma * k);
        R.tf.bias = (float)(-(double)tf->v0 * k);
    } else {
        R.tf.n = 2;
    }
    camera_setup(cam, p.width, p.height, R.cam);
    R.out = (float*)out;
    R.W = p.width;
    R.H = p.height;
    R.tiles_x = (p.width + VR_TW - 1) / VR_TW;
    R.tiles_y = (p.height + VR_TH - 1) / VR_TH;
    R.box_bytes = vr_box_bytes(p.mode == VR_EA ? tf->n : 0);
    R.mode = p.mode;
    R.interp = p.interp;
    R.use_skip = p.use_skip;
    R.step = ff{p.step, 0.0f};
    R.ert_T = p.ert_alpha > 1.0f ? -1.0f : (float)(1.0 - (double)p.ert_alpha);
    R.out_scale = (float)cube->sigma;
    if (p.use_skip) {
        MaskEntry* me = nullptr;
        vr_status st = get_mask(c, cube, p.mode, tf, clip_s, s, &me, !prepared_only);
        if (st != VR_OK) return st;
        R.cube.mask = (const uint64_t*)me->buf.ptr;
        R.cube.cellbits = (const uint32_t*)me->bits.ptr;
        R.cube.cellmax = p.mode == VR_MIP ? (const float*)me->cellmax.ptr : nullptr;
        if (mask_used) *mask_used = me;
    }
    return VR_OK;
}

vr_status mark_use(Ctx* c, Cube* cube, Tf* tf, MaskEntry* mask, hipStream_t s) {
    (void)c;
    vr_status st = cube->uses.record(s);
    if (st == VR_OK && mask) st = mask->uses.record(s);
    if (st == VR_OK && tf) st = tf->uses.record(s);
    return st;
}

static vr_status ensure_counters(Ctx* c, int count) {
    if (c->counters_cap >= count) return VR_OK;
    if (c->counters.ptr) {
        vr_status st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (st != VR_OK) return st;
        dev_free(c, c->counters, false);
    }
    int cap = std::max(count, 64);
    vr_status st = dev_alloc(c, c->counters, (uint64_t)cap * sizeof(DevCounters), false);
    if (st != VR_OK) return st;
    c->counters_cap = cap;
    return VR_OK;
}

// Dispatch-order scratch of a single render; a render on another stream waits
// for the last one that read it.
// The two order buffers of single renders (and the side stream and events),
// grown to ntiles; growing waits for the device.
static vr_status ensure_order2(Ctx* c, int ntiles) {
    vr_status st = VR_OK;
    if (!c->order_side) {
        st = hip_check(hipStreamCreateWithFlags(&c->order_side, hipStreamNonBlocking), "hipStreamCreate");
        if (st != VR_OK) {
            c->order_side = nullptr;
            return st;
        }
    }
    for (hipEvent_t* e : {&c->order2_free[0], &c->order2_free[1], &c->order2_ready})
        if (!*e) {
            st = hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
            if (st != VR_OK) {
                *e = nullptr;
                return st;
            }
        }
    if (c->order2_cap < ntiles) {
        st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (st != VR_OK) return st;
        for (int q = 0; q < 2; ++q) dev_free(c, c->order2[q], false);
        c->order2_cap = 0;
        c->order2_used[0] = c->order2_used[1] = false;
        const int cap = std::max(ntiles, 4096);
        for (int q = 0; q < 2; ++q) {
            st = dev_alloc(c, c->order2[q], (uint64_t)cap * sizeof(int) + 1024, false);
            if (st != VR_OK) return st;
        }
        c->order2_cap = cap;
    }
    return VR_OK;
}

static vr_status ensure_order(Ctx* c, int ntiles, hipStream_t s) {
    vr_status st = VR_OK;
    if (c->order_cap < ntiles) {
        if (c->order.ptr) {
            st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
            if (st != VR_OK) return st;
            dev_free(c, c->order, false);
        }
        c->order_cap = 0;
        const int cap = std::max(ntiles, 4096);
        st = dev_alloc(c, c->order, (uint64_t)cap * sizeof(int), false);
        if (st != VR_OK) return st;
        c->order_cap = cap;
    }
    if (!c->ohist.ptr) {
        st = dev_alloc(c, c->ohist, 1024, false);
        if (st != VR_OK) return st;
    }
    if (!c->order_done) {
        st = hip_check(hipEventCreateWithFlags(&c->order_done, hipEventDisableTiming), "hipEventCreate");
        if (st != VR_OK) return st;
    } else {
        st = hip_check(hipStreamWaitEvent(s, c->order_done, 0), "hipStreamWaitEvent");
    }
    return st;
}

static void fill_stats(const DevCounters& d, float ms, vr_stats* st) {
    st->samples_nominal = d.samples_nominal;
    st->samples_exec = d.samples_exec;
    st->rays_hit = d.rays_hit;
    st->rays_ert = d.rays_ert;
    st->cells_skipped = d.cells_skipped;
    st->kernel_ms = ms;
    st->reserved = 0.0f;
}

vr_status check_request(Ctx* c, const vr_request* r) {
    if (!r) {
        set_error("request is NULL");
        return VR_EINVAL;
    }
    vr_status st = check_params(&r->params);
    if (st != VR_OK) return st;
    st = check_camera(&r->camera);
    if (st != VR_OK) return st;
    if (!r->out_dev) {
        set_error("request output pointer is NULL");
        return VR_EINVAL;
    }
    if (std::isnan(r->clip)) {
        set_error("clip must not be NaN");
        return VR_EINVAL;
    }
    if (!find_cube(c, r->cube)) {
        set_error("unknown cube handle " + std::to_string(r->cube));
        return VR_ENOTFOUND;
    }
    if (r->params.mode == VR_EA) {
        const vr_tf t = r->tf ? r->tf : c->current_tf;
        if (!t) {
            set_error("no transfer function set");
            return VR_ESTATE;
        }
        if (!find_tf(c, t)) {
            set_error("unknown transfer function handle " + std::to_string(t));
            return VR_ENOTFOUND;
        }
    }
    return VR_OK;
}

void free_batch_bufs(Ctx* c, BatchBufs& bb) {
    for (auto& kv : bb.graphs) (void)hipGraphExecDestroy(kv.second);
    bb.graphs.clear();
    dev_free(c, bb.reqs, false);
    dev_free(c, bb.items, false);
    dev_free(c, bb.head, false);
    dev_free(c, bb.hdr, false);
    dev_free(c, bb.sorted, false);
    if (bb.pin_reqs) (void)hipHostFree(bb.pin_reqs);
    if (bb.pin_items) (void)hipHostFree(bb.pin_items);
    if (bb.pin_hdr) (void)hipHostFree(bb.pin_hdr);
    bb.pin_reqs = nullptr;
    bb.pin_items = nullptr;
    bb.pin_hdr = nullptr;
    bb.reqs_cap = bb.items_cap = 0;
    if (bb.done) (void)hipEventDestroy(bb.done);
    bb.done = nullptr;
}

static int pow2_at_least(int v, int lo) {
    int p = lo;
    while (p < v) p <<= 1;
    return p;
}

static vr_status grow_batch(Ctx* c, BatchBufs& bb, int nreq, int nitems) {
    g_stage = "batch buffers";
    vr_status st = ensure_event(bb.done);
    if (st != VR_OK) return st;
    // staging may still feed a queued copy
    st = hip_check(hipEventSynchronize(bb.done), "hipEventSynchronize");
    if (st != VR_OK) return st;
    if (!bb.head.ptr) {
        st = dev_alloc(c, bb.head, 256, false);
        if (st == VR_OK) st = dev_alloc(c, bb.hdr, 256, false);
        if (st == VR_OK)
            st = hip_check(hipHostMalloc((void**)&bb.pin_hdr, 256, 0), "hipHostMalloc");
        if (st != VR_OK) return st;
    }
    bool regrown = false;
    if (bb.reqs_cap < nreq) {
        const int cap = pow2_at_least(nreq, 64);
        dev_free(c, bb.reqs, false);
        if (bb.pin_reqs) (void)hipHostFree(bb.pin_reqs);
        bb.pin_reqs = nullptr;
        bb.reqs_cap = 0;
        st = dev_alloc(c, bb.reqs, (uint64_t)cap * sizeof(DevReq), false);
        if (st != VR_OK) return st;
        st = hip_check(hipHostMalloc((void**)&bb.pin_reqs, (size_t)cap * sizeof(DevReq), 0),
                       "hipHostMalloc");
        if (st != VR_OK) return st;
        bb.reqs_cap = cap;
        regrown = true;
    }
    if (bb.items_cap < nitems) {
        const int cap = pow2_at_least(nitems, 4096);
        dev_free(c, bb.items, false);
        dev_free(c, bb.sorted, false);
        if (bb.pin_items) (void)hipHostFree(bb.pin_items);
        bb.pin_items = nullptr;
        bb.items_cap = 0;
        st = dev_alloc(c, bb.items, (uint64_t)cap * sizeof(DevItem), false);
        if (st == VR_OK) st = dev_alloc(c, bb.sorted, (uint64_t)cap * sizeof(DevItem), false);
        if (st != VR_OK) return st;
        st = hip_check(hipHostMalloc((void**)&bb.pin_items, (size_t)cap * sizeof(DevItem), 0),
                       "hipHostMalloc");
        if (st != VR_OK) return st;
        bb.items_cap = cap;
        regrown = true;
    }
    if (regrown) {
        // captured graphs point at the old buffers
        for (auto& kv : bb.graphs) (void)hipGraphExecDestroy(kv.second);
        bb.graphs.clear();
    }
    return VR_OK;
}

static int log2_of(int v) {
    int k = 0;
    while ((1 << k) < v) ++k;
    return k;
}

// copies + ordering + one persistent launch per batch class present, either
// enqueued directly or captured once per (buffer sizes, LDS, classes)
static vr_status enqueue_batch(Ctx* c, BatchBufs& bb, int count, int nitems, size_t lds,
                               unsigned class_mask, DevCounters* dev_counters, hipStream_t s,
                               bool use_graph) {
    const size_t rq_bytes = (size_t)(use_graph ? bb.reqs_cap : count) * sizeof(DevReq);
    const size_t it_bytes = (size_t)(use_graph ? bb.items_cap : nitems) * sizeof(DevItem);
    const int slots = c->num_cu * VR_WG_PER_CU;  // resident workgroups
    const int grid = use_graph ? slots : std::max(1, std::min(nitems, slots));
    g_stage = "batch enqueue";
    auto record = [&]() -> vr_status {
        vr_status st = hip_check(hipMemcpyAsync(bb.hdr.ptr, bb.pin_hdr, (3 + VR_NCLASS) * sizeof(int),
                                                hipMemcpyHostToDevice, s),
                                 "hipMemcpyAsync");
        if (st == VR_OK)
            st = hip_check(hipMemcpyAsync(bb.reqs.ptr, bb.pin_reqs, rq_bytes, hipMemcpyHostToDevice, s),
                           "hipMemcpyAsync");
        if (st == VR_OK)
            st = hip_check(hipMemcpyAsync(bb.items.ptr, bb.pin_items, it_bytes, hipMemcpyHostToDevice, s),
                           "hipMemcpyAsync");
        if (st == VR_OK)
            st = hip_check(vr_launch_batch((const DevReq*)bb.reqs.ptr, (const DevItem*)bb.items.ptr,
                                           (const int*)bb.hdr.ptr, use_graph ? bb.reqs_cap : count,
                                           class_mask, (DevItem*)bb.sorted.ptr, (unsigned*)bb.head.ptr,
                                           dev_counters, lds, grid, s),
                           "batch launch");
        return st;
    };
    if (!use_graph) return record();
    // capacities are powers of two, LDS < 2^20 bytes
    const uint64_t key = ((uint64_t)log2_of(bb.items_cap) << 40) | ((uint64_t)log2_of(bb.reqs_cap) << 34) |
                         ((uint64_t)class_mask << 20) | (uint64_t)lds;
    auto it = bb.graphs.find(key);
    if (it == bb.graphs.end()) {
        vr_status st = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal),
                                 "hipStreamBeginCapture");
        if (st != VR_OK) return st;
        st = record();
        hipGraph_t g = nullptr;
        vr_status st2 = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
        if (st == VR_OK) st = st2;
        hipGraphExec_t ex = nullptr;
        if (st == VR_OK) st = hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        if (g) (void)hipGraphDestroy(g);
        if (st != VR_OK) return st;
        it = bb.graphs.emplace(key, ex).first;
    }
    return hip_check(hipGraphLaunch(it->second, s), "hipGraphLaunch");
}

vr_status launch_requests(Ctx* c, BatchBufs& bb, const vr_request* reqs, int count,
                          const int32_t* tiles, hipStream_t s, DevCounters* dev_counters,
                          bool use_graph) {
    int nitems = 0;
    for (int r = 0; r < count; ++r) {
        const auto& p = reqs[r].params;
        const int nt = ((p.width + VR_TW - 1) / VR_TW) * ((p.height + VR_TH - 1) / VR_TH);
        nitems += tiles ? (tiles[2 * r + 1] - tiles[2 * r]) : nt;
    }
    vr_status st = grow_batch(c, bb, count, std::max(nitems, 1));
    if (st != VR_OK) return st;
    int max_tf_n = 0, k = 0;
    std::vector<MaskEntry*> used((size_t)count, nullptr);
    g_stage = "cube admission";
    std::vector<Cube*> cubes_in;  // cubes of this launch: none may evict another
    for (int r = 0; r < count; ++r) {
        Cube* cube = find_cube(c, reqs[r].cube);
        st = ensure_resident(c, cube, s, true, cubes_in);
        if (st == VR_EBUSY) {
            set_error("the cubes of this batch do not fit the memory budget together");
            st = VR_ENOMEM;
        }
        if (st != VR_OK) return st;
        if (std::find(cubes_in.begin(), cubes_in.end(), cube) == cubes_in.end()) cubes_in.push_back(cube);
    }
    g_stage = "request set-up";
    c->launch_stamp = c->mask_stamp;
    for (int r = 0; r < count; ++r) {
        const vr_request& q = reqs[r];
        Cube* cube = find_cube(c, q.cube);
        Tf* tf = q.params.mode == VR_EA ? find_tf(c, q.tf ? q.tf : c->current_tf) : nullptr;
        st = build_request(c, cube, tf, q.clip, q.camera, q.params, q.out_dev, s, bb.pin_reqs[r],
                           &used[(size_t)r]);
        if (st != VR_OK) return st;
        if (tf) max_tf_n = std::max(max_tf_n, tf->n);
    }
    // work list: the items of each batch class in one run, requests in order
    unsigned class_mask = 0u;
    for (int cls = 0; cls < VR_NCLASS; ++cls) {
        bb.pin_hdr[2 + cls] = k;
        for (int r = 0; r < count; ++r) {
            const DevReq& R = bb.pin_reqs[r];
            if (VR_BATCH_CLASS(R.mode, R.cube.dtype, R.interp) != cls) continue;
            const int t0 = tiles ? tiles[2 * r] : 0;
            const int t1 = tiles ? tiles[2 * r + 1] : R.tiles_x * R.tiles_y;
            for (int t = t0; t < t1; ++t) bb.pin_items[k++] = DevItem{r, t};
            if (t1 > t0) class_mask |= 1u << cls;
        }
    }
    bb.pin_hdr[2 + VR_NCLASS] = k;
    // shape class: the TF table size fixes the LDS split (256-row tables share one class)
    if (use_graph) max_tf_n = std::max(max_tf_n, 256);
    for (int r = 0; r < count; ++r) bb.pin_reqs[r].box_bytes = vr_box_bytes(max_tf_n);
    bb.pin_hdr[0] = nitems;
    bb.pin_hdr[1] = count;
    if (nitems > 0) {
        const size_t lds = (size_t)vr_lds_reserve(max_tf_n) + 2 * (size_t)vr_box_bytes(max_tf_n);
        st = enqueue_batch(c, bb, count, nitems, lds, class_mask, dev_counters, s, use_graph);
        if (st != VR_OK) return st;
    }
    g_stage = "batch completion";
    st = hip_check(hipEventRecord(bb.done, s), "hipEventRecord");
    if (st != VR_OK) return st;
    for (int r = 0; r < count; ++r) {
        const vr_request& q = reqs[r];
        Tf* tf = q.params.mode == VR_EA ? find_tf(c, q.tf ? q.tf : c->current_tf) : nullptr;
        st = mark_use(c, find_cube(c, q.cube), tf, used[(size_t)r], s);
        if (st != VR_OK) return st;
    }
    return VR_OK;
}

static vr_status make_tf(Ctx* c, const float* rgbk, int32_t n, float v0, float v1, Tf** out) {
    std::unique_ptr<Tf> t(new Tf());
    t->id = c->next_tf++;
    t->version = c->next_tf_version++;
    t->n = n;
    t->v0 = v0;
    t->v1 = v1;
    t->rows.assign(rgbk, rgbk + 4 * n);
    if (!c->host_only()) {
        std::vector<float> dev(8 * (size_t)n, 0.0f);
        for (int i = 0; i < n; ++i)
            for (int ch = 0; ch < 4; ++ch) {
                dev[8 * i + ch] = rgbk[4 * i + ch];
                dev[8 * i + 4 + ch] = i + 1 < n ? rgbk[4 * (i + 1) + ch] - rgbk[4 * i + ch] : 0.0f;
            }
        std::vector<int> kpos((size_t)n + 2, 0);
        for (int i = 0; i < n; ++i) kpos[i + 1] = kpos[i] + (rgbk[4 * i + 3] > 0.0f ? 1 : 0);
        kpos[n + 1] = kpos[n];
        vr_status st = dev_alloc(c, t->dev_rows, dev.size() * 4, false);
        if (st != VR_OK) return st;
        st = dev_alloc(c, t->dev_kpos, kpos.size() * 4, false);
        if (st != VR_OK) {
            dev_free(c, t->dev_rows, false);
            return st;
        }
        st = hip_check(hipMemcpy(t->dev_rows.ptr, dev.data(), dev.size() * 4, hipMemcpyHostToDevice),
                       "hipMemcpy");
        if (st == VR_OK)
            st = hip_check(hipMemcpy(t->dev_kpos.ptr, kpos.data(), kpos.size() * 4,
                                     hipMemcpyHostToDevice),
                           "hipMemcpy");
        if (st != VR_OK) {
            dev_free(c, t->dev_rows, false);
            dev_free(c, t->dev_kpos, false);
            return st;
        }
    }
    *out = t.get();
    c->tfs[t->id] = std::move(t);
    return VR_OK;
}

// Free a table's device memory once every queued use of it has completed.
static vr_status free_tf_device(Ctx* c, Tf* t) {
    vr_status st = t->uses.sync();
    if (st != VR_OK) return st;
    t->uses.destroy();
    dev_free(c, t->dev_rows, false);
    dev_free(c, t->dev_kpos, false);
    return VR_OK;
}

static vr_status release_tf(Ctx* c, Tf* t) {
    vr_status st = free_tf_device(c, t);
    if (st != VR_OK) return st;
    c->tfs.erase(t->id);
    return VR_OK;
}

// Free a cube's device memory (pool, statistics, skip masks) once every
// queued use of it has completed.
static vr_status drop_device(Ctx* c, Cube* cube) {
    for (auto& lv : cube->levels) {
        vr_status st = drop_device(c, lv.get());
        if (st != VR_OK) return st;
    }
    cube->levels.clear();
    vr_status st = cube->uses.sync();
    for (auto& m : cube->masks)
        if (st == VR_OK) st = m.uses.sync();
    if (st != VR_OK) return st;
    cube->uses.destroy();
    for (auto& m : cube->masks) {
        dev_free(c, m.buf, false);
        dev_free(c, m.bits, false);
        dev_free(c, m.cellmax, false);
        m.uses.destroy();
        if (m.ready) (void)hipEventDestroy(m.ready);
    }
    cube->masks.clear();
    dev_free(c, cube->pool, true);
    dev_free(c, cube->cellmm, true);
    for (int q = 0; q < 2; ++q) {
        dev_free(c, cube->sbuf[q], true);
        cube->sbuf_sub[q] = -1;
    }
    cube->resident = false;
    return VR_OK;
}

static vr_status release_cube(Ctx* c, Cube* cube) {
    vr_status st = drop_device(c, cube);
    if (st != VR_OK) return st;
    if (cube->host_pool) (void)hipHostFree(cube->host_pool);
    cube->host_pool = nullptr;
    c->cubes.erase(cube->id);
    return VR_OK;
}

// Brick geometry of an nx*ny*nz cube stored as `storage`.
static vr_status cube_geometry(Cube* cube, int64_t nx, int64_t ny, int64_t nz, int storage,
                               double sigma) {
    cube->nx = nx;
    cube->ny = ny;
    cube->nz = nz;
    cube->storage = storage;
    cube->sigma = sigma;
    cube->Bx = (int)((nx + VR_BRICK - 1) / VR_BRICK);
    cube->By = (int)((ny + VR_BRICK - 1) / VR_BRICK);
    cube->Bz = (int)((nz + VR_BRICK - 1) / VR_BRICK);
    const int64_t ns = (int64_t)cube->Bx * cube->By * cube->Bz;
    if (ns > (int64_t)1 << 30) {
        set_error("cube too large");
        return VR_EINVAL;
    }
    cube->nslots = (int)ns;
    cube->xch = VR_XCH(storage);
    cube->stride = ((uint64_t)VR_SLOT_ZP * VR_SLOT_YG * cube->xch * 128 + 255) & ~uint64_t(255);
    return VR_OK;
}

// Allocate a cube's pool and statistics and build its bricks from src (host or
// device memory); returns once src may be reused.  On failure nothing stays
// allocated.
static vr_status cube_fill(Ctx* c, Cube* cube, const void* src, int src_dtype, int src_on_device,
                           hipStream_t s, const float* zdiv_host = nullptr) {
    auto cleanup = [&]() {
        dev_free(c, cube->pool, true);
        dev_free(c, cube->cellmm, true);
    };
    const int64_t nx = cube->nx, ny = cube->ny, nz = cube->nz;
    vr_status st = dev_alloc(c, cube->pool, (uint64_t)cube->nslots * cube->stride, true);
    if (st == VR_OK)
        st = dev_alloc(c, cube->cellmm, (uint64_t)cube->nslots * 2 * VR_CELLS_PER_BRICK * 4, true);
    if (st != VR_OK) {
        cleanup();
        return st;
    }
    const int src_kind = src_dtype == VR_F32 ? 0 : src_dtype;
    const uint64_t selem = src_dtype == VR_F32 ? 4 : 2;
    const uint64_t plane = (uint64_t)nx * ny * selem;
    DevBuf stage, zdiv;
    if (zdiv_host) {
        st = dev_alloc(c, zdiv, (uint64_t)nz * 4, false);
        if (st == VR_OK)
            st = hip_check(hipMemcpyAsync(zdiv.ptr, zdiv_host, (size_t)nz * 4, hipMemcpyHostToDevice, s),
                           "hipMemcpyAsync");
        if (st != VR_OK) {
            (void)hipStreamSynchronize(s);
            dev_free(c, zdiv, false);
            cleanup();
            return st;
        }
    }
    if (!src_on_device) {
        // a brick layer reads planes z0 .. z0 + 33 (apron and padding, edge-clamped)
        st = dev_alloc(c, stage, plane * (uint64_t)std::min<int64_t>(nz, 2 * VR_SLOT_ZP), false);
        if (st != VR_OK) {
            (void)hipStreamSynchronize(s);
            dev_free(c, zdiv, false);
            cleanup();
            return st;
        }
    }
    for (int bz = 0; bz < cube->Bz && st == VR_OK; ++bz) {
        const int64_t z0 = (int64_t)bz * VR_BRICK;
        const int64_t z1 = std::min<int64_t>(z0 + 2 * VR_SLOT_ZP, nz);
        const void* slab = src;
        int64_t z_first = 0;
        if (!src_on_device) {
            st = hip_check(hipMemcpyAsync(stage.ptr, (const uint8_t*)src + (uint64_t)z0 * plane,
                                          (size_t)((z1 - z0) * plane), hipMemcpyHostToDevice, s),
                           "hipMemcpyAsync");
            if (st != VR_OK) break;
            slab = stage.ptr;
            z_first = z0;
        }
        st = hip_check(vr_launch_brick_build(src_kind, cube->storage, slab, nx, ny, nz, z_first, bz,
                                             cube->Bx, cube->By, (uint8_t*)cube->pool.ptr,
                                             cube->stride, cube->xch, (float*)cube->cellmm.ptr,
                                             (float)cube->sigma, (const float*)zdiv.ptr, s),
                       "brick build launch");
    }
    vr_status st2 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (stage.ptr) dev_free(c, stage, false);
    if (zdiv.ptr) dev_free(c, zdiv, false);
    if (st == VR_OK) st = st2;
    if (st != VR_OK) {
        cleanup();
        return st;
    }
    cube->resident = true;
    cube->lru = ++c->lru_clock;
    return VR_OK;
}

// Evict idle registered cubes (least recently used first; never `self` or a
// cube in `keep`) until `need` more bytes fit the budget.
static vr_status make_room(Ctx* c, uint64_t need, const Cube* self, bool may_wait,
                           const std::vector<Cube*>& keep) {
    while (c->budget && c->used + need > c->budget) {
        // the progressive loop's coarse levels (of cubes other than self) go
        // before any cube
        Cube* lv_owner = nullptr;
        for (auto& kv : c->cubes) {
            Cube* o = kv.second.get();
            if (o->levels.empty() || o == self) continue;
            bool idle = true;
            for (auto& lv : o->levels) idle = idle && lv->uses.done();
            if (idle || may_wait) {
                lv_owner = o;
                break;
            }
        }
        if (lv_owner) {
            for (auto& lv : lv_owner->levels) {
                vr_status st = drop_device(c, lv.get());
                if (st != VR_OK) return st;
            }
            lv_owner->levels.clear();
            continue;
        }
        // then the sub-cube buffers other streamed cubes keep between frames
        Cube* sb_owner = nullptr;
        for (auto& kv : c->cubes) {
            Cube* o = kv.second.get();
            if (o == self || !o->sbuf[0].ptr || o->pins > 0) continue;
            if (may_wait || o->uses.done()) {
                sb_owner = o;
                break;
            }
        }
        if (sb_owner) {
            vr_status st = sb_owner->uses.sync();
            if (st != VR_OK) return st;
            for (int q = 0; q < 2; ++q) {
                dev_free(c, sb_owner->sbuf[q], true);
                sb_owner->sbuf_sub[q] = -1;
            }
            continue;
        }
        Cube* victim = nullptr;
        bool waiting = false;  // some candidate is idle but for work in flight
        for (auto& kv : c->cubes) {
            Cube* o = kv.second.get();
            if (o == self || !o->resident || !o->host_src || o->pins > 0) continue;
            if (std::find(keep.begin(), keep.end(), o) != keep.end()) continue;
            if (!may_wait && !o->uses.done()) {
                waiting = true;
                continue;
            }
            if (!victim || o->lru < victim->lru) victim = o;
        }
        if (!victim) {
            if (waiting || !keep.empty()) {
                set_error("cube does not fit the memory budget while other work holds it");
                return VR_EBUSY;
            }
            bool pinned = false;
            for (auto& kv : c->cubes) pinned = pinned || (kv.second->resident && kv.second->pins > 0);
            set_error("cube of " + std::to_string(need) + " bytes does not fit the memory budget (" +
                      std::to_string(c->used) + " of " + std::to_string(c->budget) +
                      " bytes held by cubes that cannot be evicted now)");
            return pinned ? VR_EBUSY : VR_ENOMEM;
        }
        vr_status st = drop_device(c, victim);
        if (st != VR_OK) return st;
        ++c->evictions;
    }
    return VR_OK;
}

// Brick a registered cube that exceeds the budget into pinned host memory, one
// brick layer at a time on the device, keeping only its cell statistics there.
static vr_status prepare_streamed(Ctx* c, Cube* cube, hipStream_t s) {
    const uint64_t spl = (uint64_t)cube->Bx * cube->By;  // slots per brick layer
    const uint64_t layer = spl * cube->stride;
    vr_status st = make_room(c, alloc_size((uint64_t)cube->nslots * 2 * VR_CELLS_PER_BRICK * 4), cube,
                             true, {});
    if (st == VR_OK)
        st = dev_alloc(c, cube->cellmm, (uint64_t)cube->nslots * 2 * VR_CELLS_PER_BRICK * 4, true);
    if (st != VR_OK) return st;
    if (!cube->host_pool) {
        st = hip_check(hipHostMalloc(&cube->host_pool, (size_t)(cube->nslots * cube->stride), 0),
                       "hipHostMalloc");
        if (st != VR_OK) {
            cube->host_pool = nullptr;
            dev_free(c, cube->cellmm, true);
            return st;
        }
    }
    const int64_t nx = cube->nx, ny = cube->ny, nz = cube->nz;
    const uint64_t selem = cube->src_dtype == VR_F32 ? 4 : 2;
    const uint64_t plane = (uint64_t)nx * ny * selem;
    DevBuf lbuf, stage;
    st = dev_alloc(c, lbuf, layer, false);
    if (st == VR_OK) st = dev_alloc(c, stage, plane * (uint64_t)std::min<int64_t>(nz, 2 * VR_SLOT_ZP), false);
    const int src_kind = cube->src_dtype == VR_F32 ? 0 : cube->src_dtype;
    for (int bz = 0; bz < cube->Bz && st == VR_OK; ++bz) {
        const int64_t z0 = (int64_t)bz * VR_BRICK;
        const int64_t z1 = std::min<int64_t>(z0 + 2 * VR_SLOT_ZP, nz);
        st = hip_check(hipMemcpyAsync(stage.ptr, (const uint8_t*)cube->host_src + (uint64_t)z0 * plane,
                                      (size_t)((z1 - z0) * plane), hipMemcpyHostToDevice, s),
                       "hipMemcpyAsync");
        // the layer buffer stands for slots bz*spl .. (bz+1)*spl - 1 of the pool
        uint8_t* vbase = (uint8_t*)((uintptr_t)lbuf.ptr - (uintptr_t)((uint64_t)bz * layer));
        if (st == VR_OK)
            st = hip_check(vr_launch_brick_build(src_kind, cube->storage, stage.ptr, nx, ny, nz, z0, bz,
                                                 cube->Bx, cube->By, vbase, cube->stride, cube->xch,
                                                 (float*)cube->cellmm.ptr, (float)cube->sigma, nullptr, s),
                           "brick build launch");
        if (st == VR_OK)
            st = hip_check(hipMemcpyAsync((uint8_t*)cube->host_pool + (uint64_t)bz * layer, lbuf.ptr,
                                          (size_t)layer, hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync");
        if (st == VR_OK) st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    (void)hipStreamSynchronize(s);
    dev_free(c, lbuf, false);
    dev_free(c, stage, false);
    if (st != VR_OK) {
        dev_free(c, cube->cellmm, true);
        return st;
    }
    cube->streamed = true;
    ++c->uploads;
    return VR_OK;
}

vr_status ensure_resident(Ctx* c, Cube* cube, hipStream_t s, bool may_wait,
                          const std::vector<Cube*>& keep) {
    if (cube->resident) {
        cube->lru = ++c->lru_clock;
        return VR_OK;
    }
    if (cube->host_src && c->budget && cube->need_bytes() > c->budget) {
        if (cube->streamed) return VR_OK;
        if (!may_wait || !keep.empty()) {
            set_error("a cube larger than the memory budget is rendered only by vr_render");
            return VR_EUNSUPPORTED;
        }
        return prepare_streamed(c, cube, s);
    }
    vr_status st = make_room(c, cube->need_bytes(), cube, may_wait, keep);
    if (st != VR_OK) return st;
    st = cube_fill(c, cube, cube->host_src, cube->src_dtype, 0, s);
    if (st != VR_OK) return st;
    ++c->uploads;
    return VR_OK;
}

}  // namespace vrh

using namespace vrh;

// no C++ exception crosses the C interface
#define VR_GUARD(...)                                           \
    try {                                                       \
        __VA_ARGS__                                             \
    } catch (const std::bad_alloc&) {                           \
        set_error("host allocation failed");                    \
        return VR_ENOMEM;                                       \
    } catch (const std::exception& ex) {                        \
        set_error(std::string("internal error in ") + g_stage +  \
                  ": " + ex.what());                            \
        return VR_EINVAL;                                       \
    } catch (...) {                                             \
        set_error("internal error");                            \
        return VR_EINVAL;                                       \
    }

extern "C" {

const char* vr_last_error(void) { return g_err.c_str(); }

const char* vr_version(void) { return "vr-mi355x 0.1 (gfx950)"; }

vr_status vr_create(int32_t device, uint64_t hbm_budget_bytes, const vr_allocator* alloc,
                    vr_ctx* out) {
    if (!out) {
        set_error("out is NULL");
        return VR_EINVAL;
    }
    *out = nullptr;
    if (device < -1) {
        set_error("device must be >= 0, or -1 for a host-only context");
        return VR_EINVAL;
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        set_error("allocator needs both alloc and free");
        return VR_EINVAL;
    }
    VR_GUARD({
        std::unique_ptr<Ctx> c(new Ctx());
        c->device = device;
        c->budget = hbm_budget_bytes;
        if (alloc) {
            c->has_alloc = true;
            c->alloc = *alloc;
        }
        if (device >= 0) {
            int n = 0;
            vr_status st = hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
            if (st != VR_OK) return st;
            if (device >= n) {
                set_error("device index out of range");
                return VR_EINVAL;
            }
            st = hip_check(hipSetDevice(device), "hipSetDevice");
            if (st != VR_OK) return st;
            hipDeviceProp_t prop;
            st = hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
            if (st != VR_OK) return st;
            c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
            st = noalloc_setup(device);
            if (st != VR_OK) return st;
        }
        *out = (vr_ctx)c.release();
        return VR_OK;
    });
}

vr_status vr_destroy(vr_ctx ctx) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        if (c->server) server_stop(c);
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->host_only()) {
            (void)hipSetDevice(c->device);
            (void)hipDeviceSynchronize();
            std::vector<Cube*> cs;
            for (auto& kv : c->cubes) cs.push_back(kv.second.get());
            for (Cube* cu : cs) release_cube(c, cu);
            std::vector<Tf*> ts;
            for (auto& kv : c->tfs) ts.push_back(kv.second.get());
            for (Tf* t : ts) release_tf(c, t);
            for (auto& kv : c->prog.level_tfs) free_tf_device(c, kv.second.get());
            c->prog.level_tfs.clear();
            dev_free(c, c->counters, false);
            dev_free(c, c->order, false);
            dev_free(c, c->ohist, false);
            for (int q = 0; q < 2; ++q) {
                dev_free(c, c->order2[q], false);
                if (c->order2_free[q]) (void)hipEventDestroy(c->order2_free[q]);
            }
            if (c->order2_ready) (void)hipEventDestroy(c->order2_ready);
            if (c->order_side) (void)hipStreamDestroy(c->order_side);
            dev_free(c, c->prog.low, false);
            if (c->order_done) (void)hipEventDestroy(c->order_done);
            free_batch_bufs(c, c->batch);
        }
    });
    delete c;
    return VR_OK;
}

vr_status vr_cube_upload(vr_ctx ctx, const void* src, int32_t src_dtype, int32_t src_on_device,
                         int64_t nx, int64_t ny, int64_t nz, int32_t storage, double sigma_scale,
                         void* hip_stream, vr_cube* out) {
    if (!ctx || !out || !src) {
        set_error("ctx, src and out must be non-NULL");
        return VR_EINVAL;
    }
    *out = 0;
    if (nx < 2 || ny < 2 || nz < 2 || nx > 65536 || ny > 65536 || nz > 65536) {
        set_error("cube dimensions must lie in [2, 65536]");
        return VR_EINVAL;
    }
    if (storage != VR_F32 && storage != VR_F16 && storage != VR_BF16) {
        set_error("storage must be VR_F32, VR_F16 or VR_BF16");
        return VR_EINVAL;
    }
    if (src_dtype != VR_F32 && src_dtype != VR_F16 && src_dtype != VR_BF16) {
        set_error("src_dtype must be VR_F32, VR_F16 or VR_BF16");
        return VR_EINVAL;
    }
    if (src_dtype != VR_F32 && src_dtype != storage) {
        set_error("16-bit sources are stored as-is: storage must equal src_dtype");
        return VR_EUNSUPPORTED;
    }
    if (src_on_device != 0 && src_on_device != 1) {
        set_error("src_on_device must be 0 or 1");
        return VR_EINVAL;
    }
    if (!(sigma_scale > 0.0) || !std::isfinite(sigma_scale)) {
        set_error("sigma_scale must be positive and finite");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot hold cubes");
            return VR_EDEVICE;
        }
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        std::unique_ptr<Cube> cube(new Cube());
        st = cube_geometry(cube.get(), nx, ny, nz, storage, sigma_scale);
        if (st != VR_OK) return st;
        // idle registered cubes give way to an uploaded one
        st = make_room(c, cube->need_bytes(), nullptr, true, {});
        if (st == VR_EBUSY) st = VR_ENOMEM;
        if (st != VR_OK) return st;
        st = cube_fill(c, cube.get(), src, src_dtype, src_on_device, s);
        if (st != VR_OK) return st;
        cube->id = c->next_cube++;
        *out = cube->id;
        c->cubes[cube->id] = std::move(cube);
        return VR_OK;
    });
}

vr_status vr_cube_register(vr_ctx ctx, const void* src, int32_t src_dtype, int64_t nx, int64_t ny,
                           int64_t nz, int32_t storage, double sigma_scale, vr_cube* out) {
    if (!ctx || !out || !src) {
        set_error("ctx, src and out must be non-NULL");
        return VR_EINVAL;
    }
    *out = 0;
    if (nx < 2 || ny < 2 || nz < 2 || nx > 65536 || ny > 65536 || nz > 65536) {
        set_error("cube dimensions must lie in [2, 65536]");
        return VR_EINVAL;
    }
    if (storage != VR_F32 && storage != VR_F16 && storage != VR_BF16) {
        set_error("storage must be VR_F32, VR_F16 or VR_BF16");
        return VR_EINVAL;
    }
    if (src_dtype != VR_F32 && src_dtype != VR_F16 && src_dtype != VR_BF16) {
        set_error("src_dtype must be VR_F32, VR_F16 or VR_BF16");
        return VR_EINVAL;
    }
    if (src_dtype != VR_F32 && src_dtype != storage) {
        set_error("16-bit sources are stored as-is: storage must equal src_dtype");
        return VR_EUNSUPPORTED;
    }
    if (!(sigma_scale > 0.0) || !std::isfinite(sigma_scale)) {
        set_error("sigma_scale must be positive and finite");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot hold cubes");
            return VR_EDEVICE;
        }
        std::unique_ptr<Cube> cube(new Cube());
        vr_status st = cube_geometry(cube.get(), nx, ny, nz, storage, sigma_scale);
        if (st != VR_OK) return st;
        // larger than the budget: streamed, which needs the statistics plus two
        // sub-cubes of two brick layers on the device
        const uint64_t layer = (uint64_t)cube->Bx * cube->By * cube->stride;
        const uint64_t stats_bytes = alloc_size((uint64_t)cube->nslots * 2 * VR_CELLS_PER_BRICK * 4);
        if (c->budget && cube->need_bytes() > c->budget && stats_bytes + 4 * layer > c->budget) {
            set_error("cube needs at least " + std::to_string(stats_bytes + 4 * layer) +
                      " device bytes to be streamed, more than the whole budget of " +
                      std::to_string(c->budget));
            return VR_ENOMEM;
        }
        cube->host_src = src;
        cube->src_dtype = src_dtype;
        cube->id = c->next_cube++;
        *out = cube->id;
        c->cubes[cube->id] = std::move(cube);
        return VR_OK;
    });
}

vr_status vr_get_memory_stats(vr_ctx ctx, vr_memory_stats* out) {
    if (!ctx || !out) {
        set_error("ctx and out must be non-NULL");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        std::memset(out, 0, sizeof(*out));
        out->budget_bytes = c->budget;
        out->used_bytes = c->used;
        for (auto& kv : c->cubes) {
            out->cubes += 1;
            out->resident_cubes += kv.second->resident ? 1 : 0;
            out->registered_cubes += kv.second->host_src ? 1 : 0;
        }
        out->uploads = c->uploads;
        out->evictions = c->evictions;
        return VR_OK;
    });
}

vr_status vr_estimate_channel_noise(vr_ctx ctx, const float* src, int32_t src_on_device, int64_t nx,
                                    int64_t ny, int64_t nz, void* hip_stream, float* median_out,
                                    float* mad_out, float* sigma_out) {
    if (!ctx || !src) {
        set_error("ctx and src must be non-NULL");
        return VR_EINVAL;
    }
    if (nx < 1 || ny < 1 || nz < 1 || nx * ny >= ((int64_t)1 << 31) || nz > 65536) {
        set_error("channel size nx*ny must lie in [1, 2^31) and nz in [1, 65536]");
        return VR_EINVAL;
    }
    if (src_on_device != 0 && src_on_device != 1) {
        set_error("src_on_device must be 0 or 1");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot estimate on the device");
            return VR_EDEVICE;
        }
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        const uint64_t plane = (uint64_t)nx * ny;
        DevBuf out, stage;
        st = dev_alloc(c, out, (uint64_t)nz * 12, false);
        // host sources are staged a group of channels at a time (<= 256 MiB)
        const int64_t group = src_on_device ? nz
                                            : std::max<int64_t>(1, std::min<int64_t>(nz, ((int64_t)256 << 20) / (int64_t)(plane * 4)));
        if (st == VR_OK && !src_on_device) st = dev_alloc(c, stage, plane * 4 * (uint64_t)group, false);
        float* med = (float*)out.ptr;
        for (int64_t z0 = 0; z0 < nz && st == VR_OK; z0 += group) {
            const int64_t np = std::min<int64_t>(group, nz - z0);
            const float* p = src + (uint64_t)z0 * plane;
            if (!src_on_device) {
                st = hip_check(hipMemcpyAsync(stage.ptr, p, (size_t)(np * plane * 4), hipMemcpyHostToDevice, s),
                               "hipMemcpyAsync");
                p = (const float*)stage.ptr;
            }
            if (st == VR_OK)
                st = hip_check(vr_launch_channel_noise(p, (int64_t)plane, z0, (int)np, med, med + nz,
                                                       med + 2 * nz, s),
                               "noise launch");
        }
        std::vector<float> h((size_t)nz * 3);
        if (st == VR_OK)
            st = hip_check(hipMemcpyAsync(h.data(), out.ptr, h.size() * 4, hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync");
        vr_status st2 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        dev_free(c, out, false);
        dev_free(c, stage, false);
        if (st == VR_OK) st = st2;
        if (st != VR_OK) return st;
        if (median_out) std::memcpy(median_out, h.data(), (size_t)nz * 4);
        if (mad_out) std::memcpy(mad_out, h.data() + nz, (size_t)nz * 4);
        if (sigma_out) std::memcpy(sigma_out, h.data() + 2 * nz, (size_t)nz * 4);
        return VR_OK;
    });
}

vr_status vr_cube_upload_scaled(vr_ctx ctx, const float* src, int32_t src_on_device, int64_t nx,
                                int64_t ny, int64_t nz, int32_t storage, const float* channel_divisor,
                                void* hip_stream, vr_cube* out) {
    if (!ctx || !out || !src || !channel_divisor) {
        set_error("ctx, src, channel_divisor and out must be non-NULL");
        return VR_EINVAL;
    }
    *out = 0;
    if (nx < 2 || ny < 2 || nz < 2 || nx > 65536 || ny > 65536 || nz > 65536) {
        set_error("cube dimensions must lie in [2, 65536]");
        return VR_EINVAL;
    }
    if (storage != VR_F32 && storage != VR_F16 && storage != VR_BF16) {
        set_error("storage must be VR_F32, VR_F16 or VR_BF16");
        return VR_EINVAL;
    }
    if (src_on_device != 0 && src_on_device != 1) {
        set_error("src_on_device must be 0 or 1");
        return VR_EINVAL;
    }
    for (int64_t z = 0; z < nz; ++z) {
        if (!(channel_divisor[z] > 0.0f) || !std::isfinite(channel_divisor[z])) {
            set_error("channel divisor " + std::to_string(z) + " is not positive and finite");
            return VR_EINVAL;
        }
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot hold cubes");
            return VR_EDEVICE;
        }
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        std::unique_ptr<Cube> cube(new Cube());
        st = cube_geometry(cube.get(), nx, ny, nz, storage, 1.0);
        if (st != VR_OK) return st;
        st = make_room(c, cube->need_bytes(), nullptr, true, {});
        if (st == VR_EBUSY) st = VR_ENOMEM;
        if (st != VR_OK) return st;
        st = cube_fill(c, cube.get(), src, VR_F32, src_on_device, s, channel_divisor);
        if (st != VR_OK) return st;
        cube->id = c->next_cube++;
        *out = cube->id;
        c->cubes[cube->id] = std::move(cube);
        return VR_OK;
    });
}

vr_status vr_cube_release(vr_ctx ctx, vr_cube cube) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        Cube* cu = find_cube(c, cube);
        if (!cu) {
            set_error("unknown cube handle " + std::to_string(cube));
            return VR_ENOTFOUND;
        }
        if (cu->refs > 0) {
            set_error("cube is referenced by queued requests");
            return VR_EBUSY;
        }
        (void)hipSetDevice(c->device);
        return release_cube(c, cu);
    });
}

vr_status vr_cube_get_info(vr_ctx ctx, vr_cube cube, vr_cube_info* out) {
    if (!ctx || !out) {
        set_error("ctx and out must be non-NULL");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        Cube* cu = find_cube(c, cube);
        if (!cu) {
            set_error("unknown cube handle " + std::to_string(cube));
            return VR_ENOTFOUND;
        }
        std::memset(out, 0, sizeof(*out));
        out->nx = cu->nx;
        out->ny = cu->ny;
        out->nz = cu->nz;
        out->storage = cu->storage;
        out->brick = VR_BRICK;
        out->bricks_x = cu->Bx;
        out->bricks_y = cu->By;
        out->bricks_z = cu->Bz;
        out->cell = VR_CELL;
        out->sigma_scale = cu->sigma;
        out->pool_bytes = cu->pool.bytes;
        out->brick_stride = cu->stride;
        out->aux_bytes = cu->bytes() - cu->pool.bytes;
        out->pool = cu->pool.ptr;
        out->x_chunks = cu->xch;
        out->cell_minmax = (const float*)cu->cellmm.ptr;
        out->resident = cu->resident ? 1 : 0;
        out->registered = cu->host_src ? 1 : 0;
        if (!cu->resident) {
            out->pool_bytes = (uint64_t)cu->nslots * cu->stride;
            out->vmin = out->vmax = __builtin_nanf("");
            return VR_OK;
        }
        (void)hipSetDevice(c->device);
        std::vector<float> mm((size_t)cu->nslots * 2 * VR_CELLS_PER_BRICK);
        vr_status st = hip_check(hipMemcpy(mm.data(), cu->cellmm.ptr, mm.size() * 4,
                                           hipMemcpyDeviceToHost),
                                 "hipMemcpy");
        if (st != VR_OK) return st;
        float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
        for (size_t i = 0; i < mm.size(); i += 2) {
            lo = std::min(lo, mm[i]);
            hi = std::max(hi, mm[i + 1]);
        }
        out->vmin = (float)(lo * cu->sigma);
        out->vmax = (float)(hi * cu->sigma);
        return VR_OK;
    });
}

vr_status vr_set_transfer_function(vr_ctx ctx, const float* rgbk, int32_t n, float v0, float v1) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    vr_status st = check_tf(rgbk, n, v0, v1);
    if (st != VR_OK) return st;
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->host_only()) (void)hipSetDevice(c->device);
        Tf* t = nullptr;
        st = make_tf(c, rgbk, n, v0, v1, &t);
        if (st != VR_OK) return st;
        t->internal = true;
        // the previous internal table goes once no queued request holds it
        // (release waits for queued kernels that read it)
        if (c->current_tf) {
            Tf* old = find_tf(c, c->current_tf);
            if (old && old->internal && old->refs == 0) release_tf(c, old);
        }
        c->current_tf = t->id;
        return VR_OK;
    });
}

vr_status vr_set_noise_clip(vr_ctx ctx, float k, float sigma) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    if (!(sigma > 0.0f) || !std::isfinite(sigma)) {
        set_error("sigma must be positive and finite");
        return VR_EINVAL;
    }
    if (std::isnan(k) || k == __builtin_huge_valf()) {
        set_error("k must be finite or -inf");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->clip = std::isfinite(k) ? (float)((double)k * (double)sigma) : k;
    return VR_OK;
}

vr_status vr_set_camera(vr_ctx ctx, const vr_camera* cam) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    vr_status st = check_camera(cam);
    if (st != VR_OK) return st;
    Ctx* c = (Ctx*)ctx;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->camera = *cam;
    c->has_camera = true;
    return VR_OK;
}

// A cube larger than the memory budget (registered, bricked into pinned host
// memory): rendered as sub-cubes of G brick layers along z, each uploaded with
// the layer below it (the samples at its lower face read that layer's last
// plane) into one of two device buffers while the previous one renders, each
// rendered to a partial image on the whole cube's lattice, and the partials
// integrated front to back.  G is as large as two buffers within the budget
// allow.  Early termination acts within each partial.  Waits for the frame.
static vr_status render_streamed(Ctx* c, Cube* cu, Tf* tf, const vr_render_params& p, void* out_dev,
                                 hipStream_t s, vr_stats* stats) {
    const uint64_t spl = (uint64_t)cu->Bx * cu->By;
    const uint64_t layer = spl * cu->stride;
    // room for two sub-cube buffers (counting those this cube already holds):
    // idle registered cubes give way
    const uint64_t own = cu->sbuf[0].bytes + cu->sbuf[1].bytes;
    vr_status st = make_room(c, 4 * layer > own ? 4 * layer - own : 0, cu, true, {});
    if (st != VR_OK) return st;
    if ((c->budget > c->used ? c->budget - c->used : 0) + own < 4 * layer && !cu->levels.empty()) {
        // its coarse levels leave no room for two sub-cubes: they go
        for (auto& lv : cu->levels) {
            st = drop_device(c, lv.get());
            if (st != VR_OK) return st;
        }
        cu->levels.clear();
    }
    const uint64_t avail = (c->budget > c->used ? c->budget - c->used : 0) + own;
    const int G = (int)std::min<uint64_t>((uint64_t)cu->Bz, avail / (2 * layer) - 1);
    if (G < 1) {
        set_error("no room for two streamed sub-cubes within the memory budget");
        return VR_ENOMEM;
    }
    const int nsub = (cu->Bz + G - 1) / G;
    if (nsub > VR_MAX_PARTIALS) {
        set_error("cube needs more than 64 streamed sub-cubes under this budget");
        return VR_ENOMEM;
    }
    const int ch = p.mode == VR_EA ? 4 : 1;
    const uint64_t img = (uint64_t)p.width * p.height * ch * 4;
    DevBuf* buf = cu->sbuf;
    DevBuf parts;
    hipStream_t up = nullptr;
    hipEvent_t ev_up[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr}, e0 = nullptr, e1 = nullptr;
    DevCounters* dc = nullptr;
    std::vector<const float*> pp((size_t)nsub);
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (up) (void)hipStreamSynchronize(up);
        if (st != VR_OK) cu->sbuf_sub[0] = cu->sbuf_sub[1] = -1;  // contents unknown
        dev_free(c, parts, false);
        for (auto e : {ev_up[0], ev_up[1], ev_done[0], ev_done[1], e0, e1})
            if (e) (void)hipEventDestroy(e);
        if (up) (void)hipStreamDestroy(up);
    };
    if (G != cu->sbuf_G || !buf[0].ptr || !buf[1].ptr) {
        // buffers of another sub-cube size (or none): start afresh
        for (int q = 0; q < 2; ++q) {
            dev_free(c, buf[q], true);
            cu->sbuf_sub[q] = -1;
        }
        cu->sbuf_G = G;
        for (int q = 0; q < 2 && st == VR_OK; ++q) st = dev_alloc(c, buf[q], (uint64_t)(G + 1) * layer, true);
    }
    if (st == VR_OK) st = dev_alloc(c, parts, img * nsub, false);
    if (st == VR_OK) st = hip_check(hipStreamCreateWithFlags(&up, hipStreamNonBlocking), "hipStreamCreate");
    for (auto* e : {&ev_up[0], &ev_up[1], &ev_done[0], &ev_done[1]})
        if (st == VR_OK) st = hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
    if (st == VR_OK) st = hip_check(hipEventCreate(&e0), "hipEventCreate");
    if (st == VR_OK) st = hip_check(hipEventCreate(&e1), "hipEventCreate");
    if (st == VR_OK && stats) {
        st = ensure_counters(c, nsub);
        dc = (DevCounters*)c->counters.ptr;
        if (st == VR_OK)
            st = hip_check(hipMemsetAsync(dc, 0, sizeof(DevCounters) * nsub, s), "hipMemsetAsync");
    }
    if (st == VR_OK) st = hip_check(hipEventRecord(e0, s), "hipEventRecord");
    MaskEntry* me = nullptr;
    // sub-cubes in alternating order from frame to frame; each goes to the
    // buffer that already holds it, else to the one the previous sub-cube did
    // not use (at the start: the one not holding the next sub-cube)
    const bool rev = cu->sbuf_rev;
    int q_prev = -1;
    bool read_here[2] = {false, false};  // a render of this frame reads the buffer
    for (int i = 0; i < nsub && st == VR_OK; ++i) {
        const int k = rev ? nsub - 1 - i : i;
        const int b0 = k * G, b1 = std::min(b0 + G, cu->Bz), l0 = std::max(0, b0 - 1);
        int q;
        if (cu->sbuf_sub[0] == k || cu->sbuf_sub[1] == k) {
            q = cu->sbuf_sub[0] == k ? 0 : 1;
        } else if (q_prev >= 0) {
            q = 1 - q_prev;
        } else {
            q = cu->sbuf_sub[0] == (rev ? k - 1 : k + 1) ? 1 : 0;
        }
        if (cu->sbuf_sub[q] != k) {
            // the buffer's last reader in this frame must be done with it
            if (read_here[q]) st = hip_check(hipStreamWaitEvent(up, ev_done[q], 0), "hipStreamWaitEvent");
            cu->sbuf_sub[q] = -1;
            if (st == VR_OK)
                st = hip_check(hipMemcpyAsync(buf[q].ptr, (const uint8_t*)cu->host_pool + (uint64_t)l0 * layer,
                                              (size_t)((uint64_t)(b1 - l0) * layer), hipMemcpyHostToDevice, up),
                               "hipMemcpyAsync");
            if (st == VR_OK) st = hip_check(hipEventRecord(ev_up[q], up), "hipEventRecord");
            if (st == VR_OK) st = hip_check(hipStreamWaitEvent(s, ev_up[q], 0), "hipStreamWaitEvent");
            if (st == VR_OK) cu->sbuf_sub[q] = k;
        }
        q_prev = q;
        DevReq R;
        if (st == VR_OK) {
            c->launch_stamp = c->mask_stamp;
            st = build_request(c, cu, tf, c->clip, c->camera, p, (uint8_t*)parts.ptr + img * k, s, R, &me);
        }
        if (st != VR_OK) break;
        // the buffer stands for slots l0*spl .. b1*spl - 1 of the whole pool
        R.cube.pool = (const uint8_t*)((uintptr_t)buf[q].ptr - (uintptr_t)((uint64_t)l0 * layer));
        R.cube.bz_hi = b1;
        const int z_lo = b0 * VR_BRICK, z_hi = (int)std::min<int64_t>((int64_t)b1 * VR_BRICK, cu->nz);
        R.win_axis = 2;
        R.win_lo = z_lo == 0 ? -__builtin_huge_valf() : (float)z_lo - 0.5f;
        R.win_hi = z_hi == cu->nz ? __builtin_huge_valf() : (float)z_hi - 0.5f;
        R.win_vlo = std::max(0, z_lo - 1);
        R.win_vhi = z_hi;  // the last sub-cube's samples reach the top face: floor index nz - 1
        R.partial = 1;
        pp[(size_t)k] = (const float*)((uint8_t*)parts.ptr + img * k);
        st = ensure_order(c, R.tiles_x * R.tiles_y, s);
        if (st == VR_OK)
            st = hip_check(vr_launch_render(R, (int*)c->order.ptr, (unsigned*)c->ohist.ptr,
                                            dc ? dc + k : nullptr, s),
                           "render launch");
        if (st == VR_OK) st = hip_check(hipEventRecord(c->order_done, s), "hipEventRecord");
        if (st == VR_OK) st = hip_check(hipEventRecord(ev_done[q], s), "hipEventRecord");
        read_here[q] = true;
    }
    cu->sbuf_rev = !rev;
    if (st == VR_OK) {
        DevCam cam;
        camera_setup(c->camera, p.width, p.height, cam);
        st = hip_check(vr_launch_composite(pp.data(), nsub, p.mode, 2, cam, p.width, p.height,
                                           (float*)out_dev, s),
                       "composite launch");
    }
    if (st == VR_OK) st = mark_use(c, cu, tf, me, s);
    if (st == VR_OK) st = hip_check(hipEventRecord(e1, s), "hipEventRecord");
    if (st == VR_OK) st = hip_check(hipEventSynchronize(e1), "streamed render");
    if (st == VR_OK && stats) {
        float ms = 0.0f;
        st = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        std::vector<DevCounters> h((size_t)nsub);
        if (st == VR_OK)
            st = hip_check(hipMemcpy(h.data(), dc, sizeof(DevCounters) * nsub, hipMemcpyDeviceToHost),
                           "hipMemcpy");
        if (st == VR_OK) {
            DevCounters sum{};
            for (const auto& x : h) {
                sum.samples_nominal += x.samples_nominal;
                sum.samples_exec += x.samples_exec;
                sum.rays_ert += x.rays_ert;
                sum.cells_skipped += x.cells_skipped;
                sum.rays_hit = std::max(sum.rays_hit, x.rays_hit);
            }
            fill_stats(sum, ms, stats);
        }
    }
    cleanup();
    return st;
}

// A sub-cube window: voxel planes [lo, hi) along one axis.
struct SubWindow {
    int axis, lo, hi;
};

// One image of a resident, non-streamed cube with the given camera and transfer
// function (the context's clip), optionally restricted to a sub-cube window.
static vr_status render_one(Ctx* c, Cube* cu, Tf* tf, const vr_camera& cam,
                            const vr_render_params& p, void* out_dev, hipStream_t s, vr_stats* stats,
                            const SubWindow* win) {
    vr_status st = VR_OK;
    DevReq R;
    MaskEntry* me = nullptr;
    c->launch_stamp = c->mask_stamp;
    st = build_request(c, cu, tf, c->clip, cam, p, out_dev, s, R, &me);
    if (st != VR_OK) return st;
    if (win) {
        const int64_t Na = win->axis == 0 ? cu->nx : (win->axis == 1 ? cu->ny : cu->nz);
        if (win->lo < 0 || win->hi > Na || win->lo >= win->hi) {
            set_error("sub-cube planes must satisfy 0 <= lo < hi <= the axis size");
            return VR_EINVAL;
        }
        R.win_axis = win->axis;
        R.win_lo = win->lo == 0 ? -__builtin_huge_valf() : (float)win->lo - 0.5f;
        R.win_hi = win->hi == Na ? __builtin_huge_valf() : (float)win->hi - 0.5f;
        R.win_vlo = std::max(0, win->lo - 1);
        R.win_vhi = win->hi;  // the last window's samples reach the top face: floor index Na - 1
        R.partial = 1;
    }
    DevCounters* dc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        st = ensure_counters(c, 1);
        if (st != VR_OK) return st;
        dc = (DevCounters*)c->counters.ptr;
        st = hip_check(hipMemsetAsync(dc, 0, sizeof(DevCounters), s), "hipMemsetAsync");
        if (st != VR_OK) return st;
        st = hip_check(hipEventCreate(&e0), "hipEventCreate");
        if (st == VR_OK) st = hip_check(hipEventCreate(&e1), "hipEventCreate");
        if (st == VR_OK) st = hip_check(hipEventRecord(e0, s), "hipEventRecord");
        if (st != VR_OK) return st;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    st = hip_check(hipStreamIsCapturing(s, &cap), "hipStreamIsCapturing");
    if (st != VR_OK) return st;
    if (cap != hipStreamCaptureStatusNone) {
        // under capture everything stays on the caller's stream
        st = ensure_order(c, R.tiles_x * R.tiles_y, s);
        if (st != VR_OK) return st;
        st = hip_check(vr_launch_render(R, (int*)c->order.ptr, (unsigned*)c->ohist.ptr, dc, s),
                       "render launch");
        if (st == VR_OK) st = hip_check(hipEventRecord(c->order_done, s), "hipEventRecord");
    } else {
        st = ensure_order2(c, R.tiles_x * R.tiles_y);
        if (st != VR_OK) return st;
        const int q = c->order2_next;
        c->order2_next ^= 1;
        int* ord = (int*)c->order2[q].ptr;
        unsigned* hist = (unsigned*)(ord + c->order2_cap);
        // the order needs no earlier work on s, only the end of the render
        // that last read this buffer
        if (c->order2_used[q])
            st = hip_check(hipStreamWaitEvent(c->order_side, c->order2_free[q], 0), "hipStreamWaitEvent");
        if (st == VR_OK) st = hip_check(vr_launch_order(R, ord, hist, c->order_side), "order launch");
        if (st == VR_OK) st = hip_check(hipEventRecord(c->order2_ready, c->order_side), "hipEventRecord");
        if (st == VR_OK) st = hip_check(hipStreamWaitEvent(s, c->order2_ready, 0), "hipStreamWaitEvent");
        if (st == VR_OK) st = hip_check(vr_launch_render_ordered(R, ord, dc, s), "render launch");
        if (st == VR_OK) st = hip_check(hipEventRecord(c->order2_free[q], s), "hipEventRecord");
        if (st == VR_OK) c->order2_used[q] = true;
    }
    if (st != VR_OK) return st;
    st = mark_use(c, cu, tf, me, s);
    if (st != VR_OK) return st;
    if (stats) {
        st = hip_check(hipEventRecord(e1, s), "hipEventRecord");
        if (st == VR_OK) st = hip_check(hipEventSynchronize(e1), "render");
        float ms = 0.0f;
        if (st == VR_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        DevCounters h;
        if (st == VR_OK)
            st = hip_check(hipMemcpy(&h, dc, sizeof(h), hipMemcpyDeviceToHost), "hipMemcpy");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != VR_OK) return st;
        fill_stats(h, ms, stats);
    }
    return VR_OK;
}

static vr_status render_impl(vr_ctx ctx, vr_cube cube, const vr_render_params* params, void* out_dev,
                             void* hip_stream, vr_stats* stats, const SubWindow* win) {
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
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
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
        if (c->host_only()) {
            set_error("host-only context cannot render");
            return VR_EDEVICE;
        }
        st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        st = ensure_resident(c, cu, s, true, {});
        if (st != VR_OK) return st;
        if (cu->streamed) {
            if (win) {
                set_error("sub-cube renders of a streamed cube are not supported");
                return VR_EUNSUPPORTED;
            }
            return render_streamed(c, cu, tf, *params, out_dev, s, stats);
        }
        return render_one(c, cu, tf, c->camera, *params, out_dev, s, stats, win);
    });
}

vr_status vr_render(vr_ctx ctx, vr_cube cube, const vr_render_params* params, void* out_dev,
                    void* hip_stream, vr_stats* stats) {
    return render_impl(ctx, cube, params, out_dev, hip_stream, stats, nullptr);
}

vr_status vr_render_subcube(vr_ctx ctx, vr_cube cube, const vr_render_params* params, int32_t axis,
                            int32_t plane_lo, int32_t plane_hi, void* out_dev, void* hip_stream,
                            vr_stats* stats) {
    if (axis < 0 || axis > 2) {
        set_error("axis must be 0, 1 or 2");
        return VR_EINVAL;
    }
    const SubWindow w{axis, plane_lo, plane_hi};
    return render_impl(ctx, cube, params, out_dev, hip_stream, stats, &w);
}

vr_status vr_composite(vr_ctx ctx, int32_t mode, const float* const* partials, int32_t count,
                       int32_t axis, int32_t width, int32_t height, void* out_dev, void* hip_stream) {
    if (!ctx || !partials || !out_dev) {
        set_error("ctx, partials and out_dev must be non-NULL");
        return VR_EINVAL;
    }
    if ((mode != VR_EA && mode != VR_MIP) || count < 1 || count > VR_MAX_PARTIALS || axis < 0 ||
        axis > 2 || width < 1 || height < 1 || width > 16384 || height > 16384) {
        set_error("composite: mode, count (1..64), axis or image size out of range");
        return VR_EINVAL;
    }
    for (int k = 0; k < count; ++k)
        if (!partials[k]) {
            set_error("partial " + std::to_string(k) + " is NULL");
            return VR_EINVAL;
        }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot composite");
            return VR_EDEVICE;
        }
        if (mode == VR_EA && !c->has_camera) {
            set_error("camera not set (it orders the partials along each ray)");
            return VR_ESTATE;
        }
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        DevCam cam;
        std::memset(&cam, 0, sizeof(cam));
        if (c->has_camera) camera_setup(c->camera, width, height, cam);
        return hip_check(vr_launch_composite(partials, count, mode, axis, cam, width, height,
                                             (float*)out_dev, (hipStream_t)hip_stream),
                         "composite launch");
    });
}

// ---- coarse levels of the progressive loop -----------------------------------
// Level L of a cube averages 2x2x2 blocks of level L - 1 (ceil(n/2) voxels
// per axis, the last voxel of an odd axis standing in for the missing half),
// stored as float32 in the cube's stored units.  A level-L voxel (X, Y, Z) is
// centred at full-resolution position 2^L X + (2^L - 1)/2, so the camera is
// carried into level coordinates by p -> (p - (2^L - 1)/2) / 2^L, and one level
// voxel is 2^L full-resolution lengths, so the transfer function's extinction
// is scaled by 2^L (an exact power-of-two scaling of every row).

// The next coarser level of a resident cube (or level), built on stream s.
static vr_status build_level(Ctx* c, const Cube* src, std::unique_ptr<Cube>& out, hipStream_t s) {
    std::unique_ptr<Cube> lv(new Cube());
    vr_status st = cube_geometry(lv.get(), (src->nx + 1) / 2, (src->ny + 1) / 2, (src->nz + 1) / 2,
                                 VR_F32, src->sigma);
    if (st != VR_OK) return st;
    const uint64_t pool_bytes = (uint64_t)lv->nslots * lv->stride;
    const uint64_t stat_bytes = (uint64_t)lv->nslots * 2 * VR_CELLS_PER_BRICK * 4;
    if (c->budget && c->used + alloc_size(pool_bytes) + alloc_size(stat_bytes) > c->budget)
        return VR_OK;  // does not fit the budget: no level (out stays empty)
    st = dev_alloc(c, lv->pool, pool_bytes, true);
    if (st == VR_OK) st = dev_alloc(c, lv->cellmm, stat_bytes, true);
    const int64_t plane = lv->nx * lv->ny;
    const int64_t zs = std::min<int64_t>(lv->nz, 2 * VR_SLOT_ZP);  // a brick layer's planes
    DevBuf stage;
    if (st == VR_OK) st = dev_alloc(c, stage, (uint64_t)(plane * zs) * 4, false);
    DevCube dc{};
    dc.pool = (const uint8_t*)src->pool.ptr;
    dc.stride = src->stride;
    dc.nx = (int)src->nx;
    dc.ny = (int)src->ny;
    dc.nz = (int)src->nz;
    dc.bx = src->Bx;
    dc.by = src->By;
    dc.bz = src->Bz;
    dc.dtype = src->storage;
    dc.xch = src->xch;
    dc.bz_hi = src->Bz;
    for (int bz = 0; bz < lv->Bz && st == VR_OK; ++bz) {
        const int64_t z0 = (int64_t)bz * VR_BRICK;
        const int64_t z1 = std::min<int64_t>(z0 + 2 * VR_SLOT_ZP, lv->nz);
        st = hip_check(vr_launch_mip_down(dc, (int)lv->nx, (int)lv->ny, (int)z0, (int)(z1 - z0),
                                          (float*)stage.ptr, s),
                       "coarse level launch");
        // values are already in stored units: divisor 1
        if (st == VR_OK)
            st = hip_check(vr_launch_brick_build(0, VR_F32, stage.ptr, lv->nx, lv->ny, lv->nz, z0, bz,
                                                 lv->Bx, lv->By, (uint8_t*)lv->pool.ptr, lv->stride,
                                                 lv->xch, (float*)lv->cellmm.ptr, 1.0f, nullptr, s),
                           "brick build launch");
    }
    vr_status st2 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st == VR_OK) st = st2;
    dev_free(c, stage, false);
    if (st != VR_OK) {
        dev_free(c, lv->pool, true);
        dev_free(c, lv->cellmm, true);
        return st;
    }
    lv->resident = true;
    out = std::move(lv);
    return VR_OK;
}

// Level 1 of a streamed cube, built from its pinned bricks: a coarse brick
// layer's 34 planes come from fine planes [64 bz, 64 bz + 68), so three fine
// brick layers at a time are uploaded and averaged on the device.  The
// upload buffer counts against the budget while the level is built.  The
// cube's sub-cube buffers (a cache between frames) give way to the level,
// and only if the level then fits.
static vr_status build_level_streamed(Ctx* c, Cube* src, std::unique_ptr<Cube>& out,
                                      hipStream_t s) {
    std::unique_ptr<Cube> lv(new Cube());
    vr_status st = cube_geometry(lv.get(), (src->nx + 1) / 2, (src->ny + 1) / 2, (src->nz + 1) / 2,
                                 VR_F32, src->sigma);
    if (st != VR_OK) return st;
    const uint64_t layer = (uint64_t)src->Bx * src->By * src->stride;
    const int nl = std::min(3, src->Bz);
    const uint64_t pool_bytes = (uint64_t)lv->nslots * lv->stride;
    const uint64_t stat_bytes = (uint64_t)lv->nslots * 2 * VR_CELLS_PER_BRICK * 4;
    const uint64_t own = src->sbuf[0].bytes + src->sbuf[1].bytes;
    if (c->budget && c->used - own + alloc_size(pool_bytes) + alloc_size(stat_bytes) +
                             alloc_size(nl * layer) > c->budget)
        return VR_OK;  // does not fit: no level
    if (own) {
        st = src->uses.sync();
        if (st != VR_OK) return st;
        for (int q = 0; q < 2; ++q) {
            dev_free(c, src->sbuf[q], true);
            src->sbuf_sub[q] = -1;
        }
    }
    DevBuf fine, stage;
    st = dev_alloc(c, lv->pool, pool_bytes, true);
    if (st == VR_OK) st = dev_alloc(c, lv->cellmm, stat_bytes, true);
    if (st == VR_OK) st = dev_alloc(c, fine, nl * layer, true);
    const int64_t plane = lv->nx * lv->ny;
    const int64_t zs = std::min<int64_t>(lv->nz, 2 * VR_SLOT_ZP);
    if (st == VR_OK) st = dev_alloc(c, stage, (uint64_t)(plane * zs) * 4, false);
    for (int bz = 0; bz < lv->Bz && st == VR_OK; ++bz) {
        const int f0 = 2 * bz, f1 = std::min(f0 + nl, src->Bz);  // fine layers [f0, f1)
        st = hip_check(hipMemcpyAsync(fine.ptr, (const uint8_t*)src->host_pool + (uint64_t)f0 * layer,
                                      (size_t)((uint64_t)(f1 - f0) * layer), hipMemcpyHostToDevice, s),
                       "hipMemcpyAsync");
        DevCube dc{};
        // the buffer stands for slots f0*Bx*By .. f1*Bx*By - 1 of the whole pool
        dc.pool = (const uint8_t*)((uintptr_t)fine.ptr - (uintptr_t)((uint64_t)f0 * layer));
        dc.stride = src->stride;
        dc.nx = (int)src->nx;
        dc.ny = (int)src->ny;
        dc.nz = (int)src->nz;
        dc.bx = src->Bx;
        dc.by = src->By;
        dc.bz = src->Bz;
        dc.dtype = src->storage;
        dc.xch = src->xch;
        dc.bz_hi = f1;
        const int64_t z0 = (int64_t)bz * VR_BRICK;
        const int64_t z1 = std::min<int64_t>(z0 + 2 * VR_SLOT_ZP, lv->nz);
        // coarse planes [z0, z1) read fine planes [2 z0, 2 z1) (clamped to the
        // cube), all inside fine layers [f0, f1)
        if (st == VR_OK)
            st = hip_check(vr_launch_mip_down(dc, (int)lv->nx, (int)lv->ny, (int)z0, (int)(z1 - z0),
                                              (float*)stage.ptr, s),
                           "coarse level launch");
        if (st == VR_OK)
            st = hip_check(vr_launch_brick_build(0, VR_F32, stage.ptr, lv->nx, lv->ny, lv->nz, z0, bz,
                                                 lv->Bx, lv->By, (uint8_t*)lv->pool.ptr, lv->stride,
                                                 lv->xch, (float*)lv->cellmm.ptr, 1.0f, nullptr, s),
                           "brick build launch");
    }
    vr_status st2 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st == VR_OK) st = st2;
    dev_free(c, fine, true);
    dev_free(c, stage, false);
    if (st != VR_OK) {
        dev_free(c, lv->pool, true);
        dev_free(c, lv->cellmm, true);
        return st;
    }
    lv->resident = true;
    out = std::move(lv);
    return VR_OK;
}

static vr_camera level_camera(const vr_camera& cam, int L) {
    const double k = (double)(1 << L), off = 0.5 * (k - 1.0);
    vr_camera o = cam;
    for (int a = 0; a < 3; ++a) {
        o.eye[a] = (cam.eye[a] - off) / k;
        o.target[a] = (cam.target[a] - off) / k;
    }
    o.ortho_w = cam.ortho_w / k;
    o.ortho_h = cam.ortho_h / k;
    return o;
}

// Level L of cube cu and the transfer function to render it with (*lc stays
// NULL where the level cannot be used: a streamed cube, an axis of fewer than
// two voxels at that level, a level that does not fit the budget, or an
// extinction that would overflow when scaled).
static vr_status level_view(Ctx* c, Cube* cu, int L, Tf* tf, hipStream_t s, Cube** lc, Tf** ltf) {
    *lc = nullptr;
    *ltf = nullptr;
    vr_status st = ensure_resident(c, cu, s, true, {});
    if (st != VR_OK) return st;
    int64_t n[3] = {cu->nx, cu->ny, cu->nz};
    for (int l = 0; l < L; ++l)
        for (auto& v : n) v = (v + 1) / 2;
    if (n[0] < 2 || n[1] < 2 || n[2] < 2) return VR_OK;
    if (tf) {
        auto key = std::make_pair(tf->version, L);
        auto it = c->prog.level_tfs.find(key);
        if (it == c->prog.level_tfs.end()) {
            std::vector<float> rows = tf->rows;
            for (int i = 0; i < tf->n; ++i) {
                rows[4 * (size_t)i + 3] *= (float)(1 << L);
                if (!std::isfinite(rows[4 * (size_t)i + 3])) return VR_OK;
            }
            // tables of earlier transfer functions are no longer needed
            for (auto jt = c->prog.level_tfs.begin(); jt != c->prog.level_tfs.end();) {
                if (jt->first.first != tf->version) {
                    st = free_tf_device(c, jt->second.get());
                    if (st != VR_OK) return st;
                    jt = c->prog.level_tfs.erase(jt);
                } else {
                    ++jt;
                }
            }
            Tf* t = nullptr;
            st = make_tf(c, rows.data(), tf->n, tf->v0, tf->v1, &t);
            if (st != VR_OK) return st;
            std::unique_ptr<Tf> own = std::move(c->tfs[t->id]);  // internal: no handle
            c->tfs.erase(t->id);
            it = c->prog.level_tfs.emplace(key, std::move(own)).first;
        }
        *ltf = it->second.get();
    }
    while ((int)cu->levels.size() < L) {
        const Cube* src = cu->levels.empty() ? cu : cu->levels.back().get();
        std::unique_ptr<Cube> lv;
        if (src == cu && cu->streamed) {
            st = build_level_streamed(c, cu, lv, s);
        } else {
            st = build_level(c, src, lv, s);
        }
        if (st != VR_OK) return st;
        if (!lv) return VR_OK;
        st = mark_use(c, const_cast<Cube*>(src), nullptr, nullptr, s);
        if (st != VR_OK) return st;
        cu->levels.push_back(std::move(lv));
    }
    *lc = cu->levels[(size_t)L - 1].get();
    cu->lru = ++c->lru_clock;
    return VR_OK;
}

vr_status vr_render_progressive(vr_ctx ctx, vr_cube cube, const vr_render_params* params,
                                double budget_ms, int32_t max_level, void* out_dev,
                                void* hip_stream, vr_progressive_info* info) {
    if (!ctx || !info) {
        set_error("ctx and info must be non-NULL");
        return VR_EINVAL;
    }
    std::memset(info, 0, sizeof(*info));
    vr_status st = check_params(params);
    if (st != VR_OK) return st;
    if (!out_dev) {
        set_error("out_dev is NULL");
        return VR_EINVAL;
    }
    if (max_level < 0 || max_level > VR_PROG_LEVELS - 1 || !std::isfinite(budget_ms)) {
        set_error("max_level must lie in [0, 4] and budget_ms must be finite");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (c->host_only()) {
            set_error("host-only context cannot render");
            return VR_EDEVICE;
        }
        if (!c->has_camera) {
            set_error("camera not set");
            return VR_ESTATE;
        }
        if (params->mode == VR_EA && !c->current_tf) {
            set_error("transfer function not set");
            return VR_ESTATE;
        }
        if (!find_cube(c, cube)) {
            set_error("unknown cube handle " + std::to_string(cube));
            return VR_ENOTFOUND;
        }
        // the view: everything that decides the image
        std::vector<uint8_t> key;
        auto put = [&](const void* p, size_t n) {
            key.insert(key.end(), (const uint8_t*)p, (const uint8_t*)p + n);
        };
        int64_t tfv = params->mode == VR_EA ? find_tf(c, c->current_tf)->version : -1;
        put(&cube, sizeof(cube));
        put(params, sizeof(*params));
        put(&c->camera, sizeof(c->camera));
        put(&tfv, sizeof(tfv));
        put(&c->clip, sizeof(c->clip));
        put(&out_dev, sizeof(out_dev));
        auto& P = c->prog;
        const bool same = P.valid && P.key == key;
        if (same && P.level == 0) {
            info->converged = 1;
            return VR_OK;
        }
        int L = 0;
        if (same) {
            L = P.level - 1;  // refine the view already shown
        } else if (budget_ms > 0.0) {
            // the finest level whose predicted time fits the budget; a level is
            // about 8x cheaper than the next finer one (rays / 4, samples / 2)
            L = max_level;
            if (P.ms_per_sample > 0.0 && P.last_samples > 0) {
                double pred0 = P.ms_per_sample * (double)P.last_samples;
                for (int l = 0; l <= max_level; ++l) {
                    if (pred0 / std::pow(8.0, l) <= budget_ms) {
                        L = l;
                        break;
                    }
                }
            }
        }
        L = std::min(L, max_level);
        const int ch = params->mode == VR_EA ? 4 : 1;
        vr_render_params lp = *params;
        lp.width = std::max(1, (params->width + (1 << L) - 1) >> L);
        lp.height = std::max(1, (params->height + (1 << L) - 1) >> L);
        hipStream_t s = (hipStream_t)hip_stream;
        st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        // a coarse level renders the averaged cube; where that cannot be used,
        // the full cube with a lattice step 2^L times longer
        Cube* lc = nullptr;
        Tf* ltf = nullptr;
        if (L > 0) {
            Tf* tf = params->mode == VR_EA ? find_tf(c, c->current_tf) : nullptr;
            st = level_view(c, find_cube(c, cube), L, tf, s, &lc, &ltf);
            if (st != VR_OK) return st;
        }
        if (!lc) lp.step = params->step * (float)(1 << L);
        void* target = out_dev;
        if (L > 0) {
            const uint64_t need = (uint64_t)lp.width * lp.height * ch * 4;
            if (P.low.bytes < need) {
                st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
                if (st != VR_OK) return st;
                dev_free(c, P.low, false);
                st = dev_alloc(c, P.low, need, false);
                if (st != VR_OK) return st;
            }
            target = P.low.ptr;
        }
        vr_stats rs;
        if (lc)
            st = render_one(c, lc, ltf, level_camera(c->camera, L), lp, target, s, &rs, nullptr);
        else
            st = vr_render(ctx, cube, &lp, target, hip_stream, &rs);
        if (st != VR_OK) return st;
        float ms = rs.kernel_ms;
        if (L > 0) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            st = hip_check(hipEventCreate(&e0), "hipEventCreate");
            if (st == VR_OK) st = hip_check(hipEventCreate(&e1), "hipEventCreate");
            if (st == VR_OK) st = hip_check(hipEventRecord(e0, s), "hipEventRecord");
            if (st == VR_OK)
                st = hip_check(vr_launch_upsample((const float*)P.low.ptr, lp.width, lp.height, ch,
                                                  (float*)out_dev, params->width, params->height, L, s),
                               "upsample launch");
            if (st == VR_OK) st = hip_check(hipEventRecord(e1, s), "hipEventRecord");
            if (st == VR_OK) st = hip_check(hipEventSynchronize(e1), "upsample");
            float up = 0.0f;
            if (st == VR_OK) st = hip_check(hipEventElapsedTime(&up, e0, e1), "hipEventElapsedTime");
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (st != VR_OK) return st;
            ms += up;
        }
        // running estimate of device time per nominal sample
        if (rs.samples_nominal > 0) {
            const double m = (double)rs.kernel_ms / (double)rs.samples_nominal;
            P.ms_per_sample = P.ms_per_sample > 0.0 ? 0.5 * (P.ms_per_sample + m) : m;
            P.last_samples = (uint64_t)((double)rs.samples_nominal * std::pow(8.0, L));
        }
        info->predicted_ms = P.ms_per_sample > 0.0
                                 ? (float)(P.ms_per_sample * (double)P.last_samples / std::pow(8.0, L))
                                 : 0.0f;
        P.key = key;
        P.level = L;
        P.valid = true;
        info->level = L;
        info->level_cube = lc ? 1 : 0;
        info->ms = ms;
        info->samples_nominal = rs.samples_nominal;
        return VR_OK;
    });
}

vr_status vr_tf_create(vr_ctx ctx, const float* rgbk, int32_t n, float v0, float v1, vr_tf* out) {
    if (!ctx || !out) {
        set_error("ctx and out must be non-NULL");
        return VR_EINVAL;
    }
    *out = 0;
    vr_status st = check_tf(rgbk, n, v0, v1);
    if (st != VR_OK) return st;
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->host_only()) (void)hipSetDevice(c->device);
        Tf* t = nullptr;
        st = make_tf(c, rgbk, n, v0, v1, &t);
        if (st != VR_OK) return st;
        *out = t->id;
        return VR_OK;
    });
}

vr_status vr_tf_release(vr_ctx ctx, vr_tf tf) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        Tf* t = find_tf(c, tf);
        if (!t) {
            set_error("unknown transfer function handle " + std::to_string(tf));
            return VR_ENOTFOUND;
        }
        if (tf == c->current_tf) {
            set_error("the context's current transfer function cannot be released");
            return VR_EBUSY;
        }
        if (t->refs > 0) {
            set_error("transfer function is referenced by queued requests");
            return VR_EBUSY;
        }
        if (!c->host_only()) (void)hipSetDevice(c->device);
        return release_tf(c, t);
    });
}

vr_status vr_render_batch(vr_ctx ctx, const vr_request* reqs, int32_t count, void* hip_stream,
                          vr_stats* stats) {
    if (!ctx || (!reqs && count > 0)) {
        set_error("ctx and reqs must be non-NULL");
        return VR_EINVAL;
    }
    if (count < 0 || count > 4096) {
        set_error("count must lie in [0, 4096]");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    VR_GUARD({
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        for (int r = 0; r < count; ++r) {
            vr_status st = check_request(c, &reqs[r]);
            if (st != VR_OK) {
                set_error("request " + std::to_string(r) + ": " + g_err);
                return st;
            }
        }
        if (count == 0) return VR_OK;
        if (c->host_only()) {
            set_error("host-only context cannot render");
            return VR_EDEVICE;
        }
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        if (st != VR_OK) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        DevCounters* dc = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        g_stage = "batch counters";
        if (stats) {
            st = ensure_counters(c, count);
            if (st != VR_OK) return st;
            dc = (DevCounters*)c->counters.ptr;
            st = hip_check(hipMemsetAsync(dc, 0, sizeof(DevCounters) * count, s), "hipMemsetAsync");
            if (st == VR_OK) st = hip_check(hipEventCreate(&e0), "hipEventCreate");
            if (st == VR_OK) st = hip_check(hipEventCreate(&e1), "hipEventCreate");
            if (st == VR_OK) st = hip_check(hipEventRecord(e0, s), "hipEventRecord");
            if (st != VR_OK) return st;
        }
        st = launch_requests(c, c->batch, reqs, count, nullptr, s, dc);
        if (st != VR_OK) return st;
        g_stage = "batch statistics";
        if (stats) {
            st = hip_check(hipEventRecord(e1, s), "hipEventRecord");
            if (st == VR_OK) st = hip_check(hipEventSynchronize(e1), "batch render");
            float ms = 0.0f;
            if (st == VR_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            std::vector<DevCounters> h((size_t)count);
            if (st == VR_OK)
                st = hip_check(hipMemcpy(h.data(), dc, sizeof(DevCounters) * count,
                                         hipMemcpyDeviceToHost),
                               "hipMemcpy");
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (st != VR_OK) return st;
            for (int r = 0; r < count; ++r) fill_stats(h[(size_t)r], ms, &stats[r]);
        }
        return VR_OK;
    });
}

}  // extern "C"
