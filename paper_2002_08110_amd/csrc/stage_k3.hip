// Entries of the specialised six-dimensional degree-3 stage kernel.
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {

template <typename P, int OPT>
static const void *k3_fn(int role) {
  switch (role) {
    case kK3First: return reinterpret_cast<const void *>(&stage_k3_kernel<P, OPT, kK3First>);
    case kK3Last: return reinterpret_cast<const void *>(&stage_k3_kernel<P, OPT, kK3Last>);
    default: return reinterpret_cast<const void *>(&stage_k3_kernel<P, OPT, kK3General>);
  }
}

const void *stage_k3_f64(int options, int role) {
  // bit 1 (keep the FP64 input) is implied in FP64
  if (options & kOptStream) return k3_fn<double, kOptStream>(role);
  return k3_fn<double, 0>(role);
}
const void *stage_k3_f32(int options, int role) {
  switch (options & 3) {
    case 0: return k3_fn<float, 0>(role);
    case 1: return k3_fn<float, 1>(role);
    case 2: return k3_fn<float, 2>(role);
    default: return k3_fn<float, 3>(role);
  }
}

}  // namespace hd
