// Forward-mode tangent kernels (sw_grad) and the checkpointed discrete adjoint
// of NVE velocity Verlet (sw_adjoint).
#include "sw.h"
#include "sw_internal.h"

extern "C" {

int sw_grad(sw_ctx*, const float*, const float*, const sw_params*, float*, double*, double*, void*) {
  return SW_EUNSUPPORTED;
}

int sw_adjoint(sw_ctx*, const float*, const float*, const sw_params*, double, double, int, int, double,
               double, const float*, const float*, double*, float*, float*, double*, float*, float*, void*) {
  return SW_EUNSUPPORTED;
}

}  // extern "C"
