// Instantiations of the fused stage kernel for d = 6 (3 x dims + 3 v dims), float.
#include "stage_dispatch.h"

namespace hd {
const void *stage_d6_f32(int n, int rd, int lds, int sd, int opt, int ld, int list) {
  return resolve_n<6, 3, float>(n, rd, lds, sd, opt, ld, list);
}
}  // namespace hd
