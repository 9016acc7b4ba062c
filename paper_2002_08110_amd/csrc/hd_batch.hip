// Batched stepping of several solvers (placeholder until the persistent
// batch kernel lands): reports HD_ERR_UNSUPPORTED.
#include <hip/hip_runtime.h>

#include "hd.h"

extern "C" {
hd_status hd_batch_create(hd_solver *const *, int, hd_batch **out) {
  if (out) *out = nullptr;
  return HD_ERR_UNSUPPORTED;
}
hd_status hd_batch_destroy(hd_batch *) { return HD_OK; }
hd_status hd_batch_step(hd_batch *, const double *, const int *, hd_stream) { return HD_ERR_UNSUPPORTED; }
}
