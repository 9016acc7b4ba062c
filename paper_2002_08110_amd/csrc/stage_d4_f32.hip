// Instantiations of the fused stage kernel for d = 4 (2 x dims + 2 v dims), float.
#include "stage_dispatch.h"

namespace hd {
hipError_t stage_d4_f32(int n, int rd, int lds, const StageParams<float> &prm,
                         const LaunchShape &ls, hipStream_t st) {
  return dispatch_n<4, 2, float>(n, rd, lds, prm, ls, st);
}
}  // namespace hd
