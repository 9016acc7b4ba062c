// Entries of the specialised six-dimensional degree-3 stage kernel.
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {

template <typename P, int OPT>
static const void *k3_fn() {
  return reinterpret_cast<const void *>(&stage_k3_kernel<P, OPT>);
}

const void *stage_k3_f64(int options) {
  // bit 1 (keep the FP64 input) is implied in FP64
  if (options & kOptStream) return k3_fn<double, kOptStream>();
  return k3_fn<double, 0>();
}
const void *stage_k3_f32(int options) {
  switch (options & 3) {
    case 0: return k3_fn<float, 0>();
    case 1: return k3_fn<float, 1>();
    case 2: return k3_fn<float, 2>();
    default: return k3_fn<float, 3>();
  }
}

}  // namespace hd
