// vr_render_ea_bf16.hip — single-image render kernels, emission-absorption mode, bf16 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(0, 2)
