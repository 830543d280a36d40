// vr_server.h — continuous-batching request server owned by a context.
#pragma once

#include "vr_host.h"

namespace vrh {
// Stop and join the context's server thread, if any (waits for queued work).
void server_stop(Ctx* c);
}  // namespace vrh
