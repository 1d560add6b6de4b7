// Implicit-differentiation backward pass (placeholder until the kernel lands).
#include "common.h"

extern "C" fpt_status fpt_grad(fpt_handle*, const fpt_scene*, const fpt_paths*,
                               const fpt_out*, const float*, const float*,
                               float*, float*, float*, float*, void*) {
  return FPT_EUNSUPPORTED;
}
