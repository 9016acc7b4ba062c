// Launchers of the specialised six-dimensional degree-3 stage kernel.
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {

template <typename P>
static hipError_t launch_k3(const StageParams<P> &prm, unsigned grid, hipStream_t st) {
  auto fn = stage_k3_kernel<P>;
  constexpr size_t shmem = k3_lds_bytes<P>();
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), shmem, st, prm);
  return hipGetLastError();
}

hipError_t stage_k3_f64(const StageParams<double> &prm, unsigned grid, hipStream_t st) {
  return launch_k3<double>(prm, grid, st);
}
hipError_t stage_k3_f32(const StageParams<float> &prm, unsigned grid, hipStream_t st) {
  return launch_k3<float>(prm, grid, st);
}

}  // namespace hd
