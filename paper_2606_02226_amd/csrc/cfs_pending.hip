// cfs_pending.hip -- entry points declared in cfs.h whose kernels are not
// built yet: they validate nothing and report CFS_E_UNSUPPORTED.
#include "cfs.h"
#include "cfs_api_internal.hpp"

using namespace cfs;

extern "C" int cfs_splat(const cfs_system *, const cfs_run *, const cfs_image *, float, float *,
                         int32_t, void *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_splat is not available in this build");
}
extern "C" size_t cfs_splat_backward_workspace(const cfs_system *, const cfs_run *) { return 0; }
extern "C" int cfs_splat_backward(const cfs_system *, const cfs_run *, const cfs_image *, float,
                                  const float *, const float *, int32_t, float *, void *, size_t,
                                  void *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_splat_backward is not available in this build");
}
extern "C" int cfs_batch_create(const cfs_batch_item *, int32_t, const cfs_plan *, cfs_batch **) {
  return fail(CFS_E_UNSUPPORTED, "cfs_batch_create is not available in this build");
}
extern "C" int cfs_batch_run(cfs_batch *, void *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_batch_run is not available in this build");
}
extern "C" int cfs_batch_update(cfs_batch *, int32_t, const cfs_system *, void *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_batch_update is not available in this build");
}
extern "C" int cfs_batch_plan(const cfs_batch *, cfs_plan *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_batch_plan is not available in this build");
}
extern "C" void cfs_batch_destroy(cfs_batch *) {}
extern "C" int cfs_autotune(const cfs_batch_item *, int32_t, cfs_plan *, void *) {
  return fail(CFS_E_UNSUPPORTED, "cfs_autotune is not available in this build");
}
