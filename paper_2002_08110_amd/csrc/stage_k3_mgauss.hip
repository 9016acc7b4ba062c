// Entries of the mapped-cell Gauss-Legendre stage kernel in the
// six-dimensional degree-3 thread layout.
#include "stage_dispatch.h"
#include "stage_k3_mgauss.h"

namespace hd {

const void *stage_k3mg_entry(bool f32) {
  if (f32) return reinterpret_cast<const void *>(&stage_k3mg_kernel<float, kOptStream>);
  return reinterpret_cast<const void *>(&stage_k3mg_kernel<double, kOptStream>);
}

}  // namespace hd
