// vr_render_ea_f16.hip — single-image render kernels, emission-absorption mode, f16 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(0, 1)
