// Instantiations of the fused stage kernel for d = 5 (3 x dims + 2 v dims), double.
#include "stage_dispatch.h"

namespace hd {
hipError_t stage_d5_f64(int n, int rd, int lds, const StageParams<double> &prm,
                         const LaunchShape &ls, hipStream_t st) {
  return dispatch_n<5, 3, double>(n, rd, lds, prm, ls, st);
}
}  // namespace hd
