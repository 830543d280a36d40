// vr_server.cpp — continuous-batching request server (placeholder until wired).
#include "vr_server.h"

namespace vrh {
void server_stop(Ctx* c) { (void)c; }
}  // namespace vrh

using namespace vrh;

extern "C" {
vr_status vr_server_start(vr_ctx ctx, const vr_server_cfg* cfg) {
    (void)ctx; (void)cfg;
    set_error("serving is not available in this build");
    return VR_EUNSUPPORTED;
}
vr_status vr_server_stop(vr_ctx ctx) { (void)ctx; return VR_OK; }
vr_status vr_submit(vr_ctx ctx, const vr_request* req, uint64_t* ticket) {
    (void)ctx; (void)req; (void)ticket;
    set_error("serving is not available in this build");
    return VR_EUNSUPPORTED;
}
vr_status vr_poll(vr_ctx ctx, uint64_t ticket, int32_t* done) {
    (void)ctx; (void)ticket; (void)done;
    set_error("serving is not available in this build");
    return VR_EUNSUPPORTED;
}
vr_status vr_wait(vr_ctx ctx, uint64_t ticket, double timeout_s, double* latency_s) {
    (void)ctx; (void)ticket; (void)timeout_s; (void)latency_s;
    set_error("serving is not available in this build");
    return VR_EUNSUPPORTED;
}
}
