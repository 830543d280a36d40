// vr_render_mip_f32.hip — single-image render kernels, MIP mode, f32 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(1, 0)
