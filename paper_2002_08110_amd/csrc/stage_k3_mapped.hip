// Entries of the mapped-cell collocation stage kernel in the six-dimensional
// degree-3 thread layout.
#include "stage_dispatch.h"
#include "stage_k3_mapped.h"

namespace hd {

const void *stage_k3m_entry(bool f32) {
  if (f32) return reinterpret_cast<const void *>(&stage_k3m_kernel<float, kOptStream>);
  return reinterpret_cast<const void *>(&stage_k3m_kernel<double, kOptStream>);
}

}  // namespace hd
