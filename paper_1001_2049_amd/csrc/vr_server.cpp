// vr_server.cpp — continuous-batching request server.
//
// A host thread owned by the context turns queued view requests into
// persistent batched launches (k_render_batch over a (request, tile) work
// list).  Up to max_inflight launches are in flight, each on its own stream
// with its own staging buffers; whenever one completes, the next launch is
// formed from whatever is queued at that moment, so requests that arrive
// while others are on the device join the next launch (iteration-level
// scheduling).  A request's tiles may be split over several launches (at most
// max_batch_tiles per launch), so a large image never blocks small ones for
// long.  The copies and kernels of a launch are replayed from a graph
// captured once per shape class (work-list capacity, request capacity, LDS
// split).  Every tile's pixels come from the same per-tile code whatever the
// batch holds, so a result is identical alone and in the mix.
//
// The paper's scheduler assigns sub-cubes to heterogeneous GPUs (Sec. 3,
// Fig. 1); on one GPU the corresponding job is this admission and batching
// of view requests.
#include "vr_server.h"

#include <chrono>
#include <cmath>
#include <cstring>

namespace vrh {

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Ticket {
    vr_request req{};
    int ntiles = 0;
    int next_tile = 0;    // tiles [0, next_tile) are assigned to launches
    int outstanding = 0;  // launches in flight holding some of its tiles
    bool done = false;
    bool pinned = false;  // holds a pin on its cube (admitted, keeps it resident)
    int bypassed = 0;     // launches formed while it waited for memory
    vr_status status = VR_OK;
    double t_arr = 0.0, t_first = -1.0, t_done = 0.0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    BatchBufs bb;
    bool busy = false;
    std::vector<uint64_t> tickets;  // tickets with tiles in the launch
};

struct Server {
    Ctx* c = nullptr;
    vr_server_cfg cfg{};
    std::thread th;
    std::mutex m;                     // tickets, pending, flags
    std::condition_variable cv;       // wakes the loop (submit, stop)
    std::condition_variable cv_done;  // wakes waiters
    std::deque<uint64_t> pending;     // tickets with unassigned tiles, FIFO
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    std::vector<Slot> slots;
    bool stop = false;
    vr_status fatal = VR_OK;
    std::string fatal_msg;
};

static int tiles_of(const vr_render_params& p) {
    return ((p.width + VR_TW - 1) / VR_TW) * ((p.height + VR_TH - 1) / VR_TH);
}

// Launches a request waiting for memory lets pass before the server stops
// forming launches until the device has drained enough to admit its cube.
#define VR_MAX_BYPASS 4

// release the cube/TF references of a finished ticket (context lock held)
static void drop_refs(Ctx* c, Ticket& tk) {
    const vr_request& r = tk.req;
    if (Cube* cu = find_cube(c, r.cube)) {
        --cu->refs;
        if (tk.pinned) --cu->pins;
    }
    tk.pinned = false;
    if (r.params.mode == VR_EA)
        if (Tf* t = find_tf(c, r.tf)) --t->refs;
}

static void fail_all(Server* S, vr_status st, const std::string& msg) {
    std::lock_guard<std::recursive_mutex> lkc(S->c->mu);
    std::lock_guard<std::mutex> lk(S->m);
    S->fatal = st;
    S->fatal_msg = msg;
    const double t = now_s();
    for (auto& kv : S->tickets) {
        if (!kv.second.done) {
            kv.second.done = true;
            kv.second.status = st;
            kv.second.t_done = t;
            drop_refs(S->c, kv.second);
        }
    }
    S->pending.clear();
    S->cv_done.notify_all();
}

static void server_loop(Server* S) {
    Ctx* c = S->c;
    (void)hipSetDevice(c->device);
    std::vector<vr_request> reqs;
    std::vector<int32_t> ranges;
    std::vector<uint64_t> ids;
    for (;;) {
        // 1. retire finished launches
        bool any_busy = false;
        for (auto& sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            if (q != hipSuccess) {
                (void)hipGetLastError();
                fail_all(S, VR_EDEVICE, std::string("device error: ") + hipGetErrorString(q));
                return;
            }
            const double t = now_s();
            std::lock_guard<std::recursive_mutex> lkc(c->mu);
            std::lock_guard<std::mutex> lk(S->m);
            for (uint64_t id : sl.tickets) {
                Ticket& tk = S->tickets[id];
                if (--tk.outstanding == 0 && tk.next_tile >= tk.ntiles && !tk.done) {
                    tk.done = true;
                    tk.t_done = t;
                    drop_refs(c, tk);
                }
            }
            sl.tickets.clear();
            sl.busy = false;
            S->cv_done.notify_all();
        }
        // 2. form launches for free slots from what is queued now.  Requests are
        // taken in arrival order; one whose cube cannot be admitted yet (memory
        // held by running work) blocks later requests that would need memory,
        // while requests for resident cubes may pass it, for VR_MAX_BYPASS
        // launches; after that no request is started until it is admitted.
        // Requests already started (their cubes pinned) always continue: they
        // hold the memory the waiting request needs.
        bool launched = false;
        bool blocked = false;
        for (auto& sl : S->slots) {
            if (sl.busy) continue;
            reqs.clear();
            ranges.clear();
            ids.clear();
            vr_status dev_err = VR_OK;
            {
                std::lock_guard<std::recursive_mutex> lkc(c->mu);
                std::lock_guard<std::mutex> lk(S->m);
                if (S->pending.empty()) break;
                int budget = S->cfg.max_batch_tiles;
                const double t = now_s();
                std::vector<Cube*> keep;
                Ticket* blocker = nullptr;
                bool start_none = false;  // the blocker has waited long enough
                auto itp = S->pending.begin();
                while (itp != S->pending.end() && budget > 0 &&
                       (int)reqs.size() < S->cfg.max_batch_requests) {
                    const uint64_t id = *itp;
                    Ticket& tk = S->tickets[id];
                    Cube* cube = find_cube(c, tk.req.cube);
                    if (!tk.pinned) {
                        if (start_none || (blocker && !cube->resident)) {
                            ++itp;  // would take memory an older request waits for
                            continue;
                        }
                        const vr_status st = ensure_resident(c, cube, sl.stream, false, keep);
                        if (st == VR_EBUSY || (st == VR_ENOMEM && !keep.empty())) {
                            if (!blocker) {
                                blocker = &tk;
                                start_none = tk.bypassed >= VR_MAX_BYPASS;
                            }
                            ++itp;
                            continue;
                        }
                        if (st == VR_ENOMEM || st == VR_EUNSUPPORTED) {
                            // can never fit beside what must stay resident, or a
                            // cube larger than the budget (streamed by vr_render only)
                            tk.done = true;
                            tk.status = st;
                            tk.t_done = t;
                            drop_refs(c, tk);
                            itp = S->pending.erase(itp);
                            S->cv_done.notify_all();
                            continue;
                        }
                        if (st != VR_OK) {
                            dev_err = st;
                            break;
                        }
                        ++cube->pins;
                        tk.pinned = true;
                    }
                    if (std::find(keep.begin(), keep.end(), cube) == keep.end()) keep.push_back(cube);
                    const int take = std::min(budget, tk.ntiles - tk.next_tile);
                    reqs.push_back(tk.req);
                    ranges.push_back(tk.next_tile);
                    ranges.push_back(tk.next_tile + take);
                    ids.push_back(id);
                    tk.next_tile += take;
                    ++tk.outstanding;
                    if (tk.t_first < 0.0) tk.t_first = t;
                    budget -= take;
                    if (tk.next_tile >= tk.ntiles) itp = S->pending.erase(itp);
                    else ++itp;
                }
                if (blocker) {
                    blocked = true;
                    if (!reqs.empty()) ++blocker->bypassed;
                }
                if (dev_err == VR_OK && !reqs.empty()) {
                    dev_err = launch_requests(c, sl.bb, reqs.data(), (int)reqs.size(), ranges.data(),
                                              sl.stream, nullptr, S->cfg.use_graphs != 0);
                    if (dev_err == VR_OK)
                        dev_err = hip_check(hipEventRecord(sl.ev, sl.stream), "hipEventRecord");
                }
            }
            if (dev_err != VR_OK) {
                fail_all(S, dev_err, "launch failed: " + std::string(vr_last_error()));
                return;
            }
            if (reqs.empty()) break;
            sl.tickets = ids;
            sl.busy = true;
            any_busy = true;
            launched = true;
        }
        // 3. sleep until there is something to do
        std::unique_lock<std::mutex> lk(S->m);
        if (S->stop && S->pending.empty() && !any_busy) break;
        if (launched) continue;
        if (any_busy) {
            S->cv.wait_for(lk, std::chrono::microseconds(20));
        } else if (blocked) {
            // memory is held by work outside the server (renders on other streams)
            S->cv.wait_for(lk, std::chrono::microseconds(500));
        } else if (S->pending.empty() && !S->stop) {
            S->cv.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        }
    }
}

void server_stop(Ctx* c) {
    std::shared_ptr<Server> S;
    {
        std::lock_guard<std::mutex> g(c->server_mu);
        S.swap(c->server);
    }
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    std::lock_guard<std::recursive_mutex> lkc(c->mu);
    (void)hipSetDevice(c->device);
    for (auto& sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        free_batch_bufs(c, sl.bb);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    // requests never completed (after a device error) still hold references
    {
        std::lock_guard<std::mutex> lk(S->m);
        for (auto& kv : S->tickets) {
            if (!kv.second.done) {
                drop_refs(c, kv.second);
                kv.second.done = true;
                kv.second.status = VR_ESTATE;
            }
        }
        if (S->fatal == VR_OK) {
            S->fatal = VR_ESTATE;
            S->fatal_msg = "server stopped";
        }
    }
    S->cv_done.notify_all();
    // callers still blocked in vr_wait hold their own reference to S
}

static std::shared_ptr<Server> get_server(Ctx* c) {
    std::lock_guard<std::mutex> g(c->server_mu);
    return c->server;
}

}  // namespace vrh

using namespace vrh;

extern "C" {

vr_status vr_server_start(vr_ctx ctx, const vr_server_cfg* cfg) {
    if (!ctx || !cfg) {
        set_error("ctx and cfg must be non-NULL");
        return VR_EINVAL;
    }
    if (cfg->max_batch_requests < 1 || cfg->max_batch_requests > 4096 || cfg->max_batch_tiles < 1 ||
        cfg->max_inflight < 1 || cfg->max_inflight > 4 ||
        (cfg->use_graphs != 0 && cfg->use_graphs != 1)) {
        set_error("server config out of range");
        return VR_EINVAL;
    }
    Ctx* c = (Ctx*)ctx;
    if (c->host_only()) {
        set_error("host-only context cannot serve");
        return VR_EDEVICE;
    }
    try {
        std::lock_guard<std::mutex> g(c->server_mu);
        if (c->server) {
            set_error("server already running");
            return VR_ESTATE;
        }
        std::unique_ptr<Server> S(new Server());
        S->c = c;
        S->cfg = *cfg;
        S->slots.resize((size_t)cfg->max_inflight);
        vr_status st = hip_check(hipSetDevice(c->device), "hipSetDevice");
        for (auto& sl : S->slots) {
            if (st != VR_OK) break;
            // default priority: streams of different priorities are avoided on purpose
            st = hip_check(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking),
                           "hipStreamCreate");
            if (st == VR_OK)
                st = hip_check(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming),
                               "hipEventCreate");
        }
        if (st != VR_OK) {
            for (auto& sl : S->slots) {
                if (sl.ev) (void)hipEventDestroy(sl.ev);
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
            }
            return st;
        }
        std::shared_ptr<Server> sp(S.release());
        sp->th = std::thread(server_loop, sp.get());
        c->server = sp;
        return VR_OK;
    } catch (const std::exception& ex) {
        set_error(std::string("server start: ") + ex.what());
        return VR_ENOMEM;
    }
}

vr_status vr_server_stop(vr_ctx ctx) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    try {
        server_stop((Ctx*)ctx);
    } catch (...) {
        set_error("server stop failed");
        return VR_EDEVICE;
    }
    return VR_OK;
}

vr_status vr_submit(vr_ctx ctx, const vr_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket) {
        set_error("ctx, req and ticket must be non-NULL");
        return VR_EINVAL;
    }
    *ticket = 0;
    Ctx* c = (Ctx*)ctx;
    std::shared_ptr<Server> S = get_server(c);
    if (!S) {
        set_error("server not running");
        return VR_ESTATE;
    }
    try {
        Ticket tk;
        tk.req = *req;
        {
            std::lock_guard<std::recursive_mutex> lkc(c->mu);
            vr_status st = check_request(c, req);
            if (st != VR_OK) return st;
            // the request keeps the transfer function current at submission
            if (tk.req.params.mode == VR_EA && tk.req.tf == 0) tk.req.tf = c->current_tf;
            ++find_cube(c, tk.req.cube)->refs;
            if (tk.req.params.mode == VR_EA) ++find_tf(c, tk.req.tf)->refs;
        }
        tk.ntiles = tiles_of(req->params);
        tk.t_arr = now_s();
        vr_status fatal = VR_OK;
        std::string fatal_msg;
        {
            std::lock_guard<std::mutex> lk(S->m);
            if (S->fatal != VR_OK) {
                fatal = S->fatal;
                fatal_msg = S->fatal_msg;
            } else {
                const uint64_t id = S->next_ticket++;
                S->tickets[id] = tk;
                S->pending.push_back(id);
                *ticket = id;
            }
        }
        if (fatal != VR_OK) {
            // lock order is context, then server: take the context lock on its own
            std::lock_guard<std::recursive_mutex> lkc(c->mu);
            drop_refs(c, tk);
            set_error("server stopped after: " + fatal_msg);
            return fatal;
        }
        S->cv.notify_one();
        return VR_OK;
    } catch (const std::exception& ex) {
        set_error(std::string("submit: ") + ex.what());
        return VR_ENOMEM;
    }
}

vr_status vr_poll(vr_ctx ctx, uint64_t ticket, int32_t* done) {
    if (!ctx || !done) {
        set_error("ctx and done must be non-NULL");
        return VR_EINVAL;
    }
    *done = 0;
    std::shared_ptr<Server> S = get_server((Ctx*)ctx);
    if (!S) {
        set_error("server not running");
        return VR_ESTATE;
    }
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        set_error("unknown ticket");
        return VR_ENOTFOUND;
    }
    *done = it->second.done ? 1 : 0;
    return it->second.done ? it->second.status : VR_OK;
}

vr_status vr_wait(vr_ctx ctx, uint64_t ticket, double timeout_s, double* latency_s) {
    if (!ctx) {
        set_error("ctx is NULL");
        return VR_EINVAL;
    }
    std::shared_ptr<Server> S = get_server((Ctx*)ctx);
    if (!S) {
        set_error("server not running");
        return VR_ESTATE;
    }
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        set_error("unknown ticket");
        return VR_ENOTFOUND;
    }
    auto pred = [&] { return S->tickets[ticket].done; };
    if (timeout_s > 0.0) {
        if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
            set_error("timed out");
            return VR_EBUSY;
        }
    } else {
        S->cv_done.wait(lk, pred);
    }
    Ticket& tk = S->tickets[ticket];
    if (latency_s) *latency_s = tk.t_done - tk.t_arr;
    const vr_status st = tk.status;
    if (st != VR_OK) set_error("request failed: " + S->fatal_msg);
    S->tickets.erase(ticket);
    return st;
}

}  // extern "C"
