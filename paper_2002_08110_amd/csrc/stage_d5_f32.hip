// Instantiations of the fused stage kernel for d = 5 (3 x dims + 2 v dims), float.
#include "stage_dispatch.h"

namespace hd {
const void *stage_d5_f32(int n, int rd, int lds, int sd, int opt, int ld, int list) {
  return resolve_n<5, 3, float>(n, rd, lds, sd, opt, ld, list);
}
}  // namespace hd
