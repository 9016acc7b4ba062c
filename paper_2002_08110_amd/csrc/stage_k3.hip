// Launchers of the specialised six-dimensional degree-3 stage kernel.
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {

template <typename P, int OPT>
static hipError_t launch_k3(const StageParams<P> &prm, unsigned grid, hipStream_t st) {
  auto fn = stage_k3_kernel<P, OPT>;
  constexpr size_t shmem = k3_lds_bytes<P>();
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), shmem, st, prm);
  return hipGetLastError();
}

hipError_t stage_k3_f64(const StageParams<double> &prm, unsigned grid, int options,
                        hipStream_t st) {
  // bit 1 (keep the FP64 input) is implied in FP64
  if (options & kOptStream) return launch_k3<double, kOptStream>(prm, grid, st);
  return launch_k3<double, 0>(prm, grid, st);
}
hipError_t stage_k3_f32(const StageParams<float> &prm, unsigned grid, int options,
                        hipStream_t st) {
  switch (options & 3) {
    case 0: return launch_k3<float, 0>(prm, grid, st);
    case 1: return launch_k3<float, 1>(prm, grid, st);
    case 2: return launch_k3<float, 2>(prm, grid, st);
    default: return launch_k3<float, 3>(prm, grid, st);
  }
}

}  // namespace hd
