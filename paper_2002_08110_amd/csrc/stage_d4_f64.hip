// Instantiations of the fused stage kernel for d = 4 (2 x dims + 2 v dims), double.
#include "stage_dispatch.h"

namespace hd {
const void *stage_d4_f64(int n, int rd, int lds, int sd, int opt, int ld, int list) {
  return resolve_n<4, 2, double>(n, rd, lds, sd, opt, ld, list);
}
}  // namespace hd
