// 3D ideal-MHD stage (placeholder until the kernel lands).
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {
hipError_t launch_cart3d(const dg_mesh*, int, const void*, const void*, void*, const double*,
                         double, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_cart3d_cfl(const dg_mesh*, const void*, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace dg
