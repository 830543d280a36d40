// vr_render_mip_bf16.hip — single-image render kernels, MIP mode, bf16 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(1, 2)
