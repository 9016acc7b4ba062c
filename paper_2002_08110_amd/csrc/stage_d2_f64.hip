// Instantiations of the fused stage kernel for d = 2 (1 x dims + 1 v dims), double.
#include "stage_dispatch.h"

namespace hd {
const void *stage_d2_f64(int n, int rd, int lds, int sd, int opt, int ld, int list) {
  return resolve_n<2, 1, double>(n, rd, lds, sd, opt, ld, list);
}
}  // namespace hd
