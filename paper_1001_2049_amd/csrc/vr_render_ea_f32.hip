// vr_render_ea_f32.hip — single-image render kernels, emission-absorption mode, f32 storage.
#include "vr_render.h"

VR_RENDER_LAUNCHER(0, 0)
