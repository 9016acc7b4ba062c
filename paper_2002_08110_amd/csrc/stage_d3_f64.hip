// Instantiations of the fused stage kernel for d = 3 (2 x dims + 1 v dims), double.
#include "stage_dispatch.h"

namespace hd {
hipError_t stage_d3_f64(int n, int rd, int lds, const StageParams<double> &prm,
                         const LaunchShape &ls, hipStream_t st) {
  return dispatch_n<3, 2, double>(n, rd, lds, prm, ls, st);
}
}  // namespace hd
