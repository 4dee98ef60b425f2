// Several events of uneven size in one persistent launch (placeholder until implemented).
#include <hip/hip_runtime.h>

#include "gwl_runtime.h"

using namespace gwl;

extern "C" {

gwl_status gwl_multi_plan_create(const gwl_event*, int, const int64_t*, gwl_precision, int, gwl_plan* out) {
  clear_error();
  if (out) *out = nullptr;
  return fail(GWL_E_UNSUPPORTED, "multi-event plans are not implemented yet");
}

gwl_status gwl_multi_launch(gwl_plan, const double* const*, double* const*, double* const*, double*, void*) {
  clear_error();
  return fail(GWL_E_UNSUPPORTED, "multi-event plans are not implemented yet");
}

gwl_status gwl_plan_destroy(gwl_plan) { return GWL_OK; }

}  // extern "C"
