// 2D face-list stage (placeholder until the kernel lands).
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {
dg_status facelist_create(dg_mesh*, const dg_mesh_desc*) {
  set_error("face-list meshes not built yet");
  return DG_EUNSUPPORTED;
}
void facelist_destroy(dg_mesh*) {}
hipError_t launch_facelist(const dg_mesh*, int, const void*, const void*, void*, const double*,
                           double, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_facelist_cfl(const dg_mesh*, const void*, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace dg
