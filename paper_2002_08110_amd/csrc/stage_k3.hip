// Entries of the specialised six-dimensional degree-3 stage kernel.
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {

template <typename P, int OPT, int ROLE>
static const void *k3_role_fn(int list) {
  if (list) return reinterpret_cast<const void *>(&stage_k3_list_kernel<P, OPT, ROLE>);
  return reinterpret_cast<const void *>(&stage_k3_kernel<P, OPT, ROLE>);
}

template <typename P, int OPT>
static const void *k3_fn(int role, int list) {
  switch (role) {
    case kK3First: return k3_role_fn<P, OPT, kK3First>(list);
    case kK3Last: return k3_role_fn<P, OPT, kK3Last>(list);
    default: return k3_role_fn<P, OPT, kK3General>(list);
  }
}

const void *stage_k3_f64(int options, int role, int list) {
  // bit 1 (keep the FP64 input) is implied in FP64
  if (options & kOptStream) return k3_fn<double, kOptStream>(role, list);
  return k3_fn<double, 0>(role, list);
}
const void *stage_k3_f32(int options, int role, int list) {
  switch (options & 3) {
    case 0: return k3_fn<float, 0>(role, list);
    case 1: return k3_fn<float, 1>(role, list);
    case 2: return k3_fn<float, 2>(role, list);
    default: return k3_fn<float, 3>(role, list);
  }
}

}  // namespace hd
