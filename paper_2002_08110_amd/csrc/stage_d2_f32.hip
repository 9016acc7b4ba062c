// Instantiations of the fused stage kernel for d = 2 (1 x dims + 1 v dims), float.
#include "stage_dispatch.h"

namespace hd {
hipError_t stage_d2_f32(int n, int rd, int lds, const StageParams<float> &prm,
                         const LaunchShape &ls, hipStream_t st) {
  return dispatch_n<2, 1, float>(n, rd, lds, prm, ls, st);
}
}  // namespace hd
