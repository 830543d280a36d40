// vr_render_mip_f16.hip — single-image render kernels, MIP mode, f16 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(1, 1)
