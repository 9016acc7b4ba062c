// Launch helpers and per-dimension dispatch of the fused stage kernel. Each
// stage_dN.hip translation unit instantiates the kernels of one dimension d
// (all degrees, both precisions, both LDS modes, the valid register-dim
// counts) so the instantiations compile in parallel.
#pragma once

#include "stage_kernel.h"

namespace hd {

constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

struct LaunchShape {
  unsigned grid, block;
  size_t shmem;
};

template <int D, int N, int DX, int RD, typename P, bool LDS>
hipError_t launch_stage(const StageParams<P> &prm, const LaunchShape &ls, hipStream_t st) {
  auto fn = stage_kernel<D, N, DX, RD, P, LDS>;
  if (ls.shmem > 65536) {
    // Once per kernel: allow the largest LDS size any plan can request.
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)kMaxLdsBytes);
    if (attr != hipSuccess) return attr;
  }
  hipLaunchKernelGGL(fn, dim3(ls.grid), dim3(ls.block), ls.shmem, st, prm);
  return hipGetLastError();
}

// True if the LDS variant of (D, N, RD, P) can hold at least one cell.
template <int D, int N, int RD, typename P>
constexpr bool lds_variant_ok() {
  return ipow(N, D - RD) <= 1024 && (size_t)ipow(N, D) * sizeof(P) <= kMaxLdsBytes;
}

template <int D, int N, int DX, int RD, typename P>
hipError_t dispatch_lds(int lds, const StageParams<P> &prm, const LaunchShape &ls,
                        hipStream_t st) {
  if (lds) {
    if constexpr (lds_variant_ok<D, N, RD, P>())
      return launch_stage<D, N, DX, RD, P, true>(prm, ls, st);
    else
      return hipErrorInvalidConfiguration;
  }
  return launch_stage<D, N, DX, RD, P, false>(prm, ls, st);
}

template <int D, int N, int DX, typename P>
hipError_t dispatch_rd(int rd, int lds, const StageParams<P> &prm, const LaunchShape &ls,
                       hipStream_t st) {
  constexpr int DV = D - DX;
  if (rd == 1) return dispatch_lds<D, N, DX, 1, P>(lds, prm, ls, st);
  if constexpr (DV >= 2) {
    if (rd == 2) return dispatch_lds<D, N, DX, 2, P>(lds, prm, ls, st);
  }
  return hipErrorInvalidConfiguration;
}

template <int D, int DX, typename P>
hipError_t dispatch_n(int n, int rd, int lds, const StageParams<P> &prm, const LaunchShape &ls,
                      hipStream_t st) {
  switch (n) {
    case 2: return dispatch_rd<D, 2, DX, P>(rd, lds, prm, ls, st);
    case 3: return dispatch_rd<D, 3, DX, P>(rd, lds, prm, ls, st);
    case 4: return dispatch_rd<D, 4, DX, P>(rd, lds, prm, ls, st);
    case 5: return dispatch_rd<D, 5, DX, P>(rd, lds, prm, ls, st);
    case 6: return dispatch_rd<D, 6, DX, P>(rd, lds, prm, ls, st);
    default: return hipErrorInvalidConfiguration;
  }
}

// Defined in stage_dN.hip (one per dimension and precision).
hipError_t stage_d2_f64(int n, int rd, int lds, const StageParams<double> &, const LaunchShape &, hipStream_t);
hipError_t stage_d3_f64(int n, int rd, int lds, const StageParams<double> &, const LaunchShape &, hipStream_t);
hipError_t stage_d4_f64(int n, int rd, int lds, const StageParams<double> &, const LaunchShape &, hipStream_t);
hipError_t stage_d5_f64(int n, int rd, int lds, const StageParams<double> &, const LaunchShape &, hipStream_t);
hipError_t stage_d6_f64(int n, int rd, int lds, const StageParams<double> &, const LaunchShape &, hipStream_t);
hipError_t stage_d2_f32(int n, int rd, int lds, const StageParams<float> &, const LaunchShape &, hipStream_t);
hipError_t stage_d3_f32(int n, int rd, int lds, const StageParams<float> &, const LaunchShape &, hipStream_t);
hipError_t stage_d4_f32(int n, int rd, int lds, const StageParams<float> &, const LaunchShape &, hipStream_t);
hipError_t stage_d5_f32(int n, int rd, int lds, const StageParams<float> &, const LaunchShape &, hipStream_t);
hipError_t stage_d6_f32(int n, int rd, int lds, const StageParams<float> &, const LaunchShape &, hipStream_t);

// Specialised kernel for d = 6 (3 x + 3 v), degree 3: one cell per
// 256-thread workgroup (stage_k3.hip).
hipError_t stage_k3_f64(const StageParams<double> &, unsigned grid, int options, hipStream_t);
hipError_t stage_k3_f32(const StageParams<float> &, unsigned grid, int options, hipStream_t);

}  // namespace hd
