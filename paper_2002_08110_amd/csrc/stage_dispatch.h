// Kernel resolution for the fused stage: from runtime (d, degree, register
// dims, LDS mode, precision) to the entry of the compiled variant. Each
// stage_dN.hip translation unit instantiates the kernels of one dimension d
// (all degrees, both precisions, both LDS modes, the valid register-dim
// counts) so the instantiations compile in parallel. The caller launches the
// returned entry with hipLaunchKernel.
#pragma once

#include "stage_kernel.h"

namespace hd {

constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

struct LaunchShape {
  unsigned grid, block;
  size_t shmem;
};

// Lets a kernel use the whole LDS of a workgroup; the entry, or nullptr if
// the runtime refuses.
inline const void *allow_max_lds(const void *fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
                 hipSuccess
             ? fn
             : nullptr;
}

// True if the LDS variant of (D, N, RD, P) can hold at least one cell.
template <int D, int N, int RD, typename P>
constexpr bool lds_variant_ok() {
  return ipow(N, D - RD) <= 1024 && (size_t)ipow(N, D) * sizeof(P) <= kMaxLdsBytes;
}

template <int D, int N, int DX, int RD, typename P, bool LDS>
const void *variant_fn() {
  static const void *const f = [] {
    const void *k = reinterpret_cast<const void *>(&stage_kernel<D, N, DX, RD, P, LDS>);
    return LDS ? allow_max_lds(k, kMaxLdsBytes) : k;
  }();
  return f;
}

template <int D, int N, int DX, int RD, typename P>
const void *resolve_lds(int lds) {
  if (lds) {
    if constexpr (lds_variant_ok<D, N, RD, P>()) return variant_fn<D, N, DX, RD, P, true>();
    else return nullptr;
  }
  return variant_fn<D, N, DX, RD, P, false>();
}

template <int D, int N, int DX, typename P>
const void *resolve_rd(int rd, int lds) {
  constexpr int DV = D - DX;
  if (rd == 1) return resolve_lds<D, N, DX, 1, P>(lds);
  if constexpr (DV >= 2) {
    if (rd == 2) return resolve_lds<D, N, DX, 2, P>(lds);
  }
  return nullptr;
}

template <int D, int DX, typename P>
const void *resolve_n(int n, int rd, int lds) {
  switch (n) {
    case 2: return resolve_rd<D, 2, DX, P>(rd, lds);
    case 3: return resolve_rd<D, 3, DX, P>(rd, lds);
    case 4: return resolve_rd<D, 4, DX, P>(rd, lds);
    case 5: return resolve_rd<D, 5, DX, P>(rd, lds);
    case 6: return resolve_rd<D, 6, DX, P>(rd, lds);
    default: return nullptr;
  }
}

// Defined in stage_dN_fP.hip (one per dimension and precision): the entry of
// the generic kernel for n = degree + 1 nodes per dimension, or nullptr.
const void *stage_d2_f64(int n, int rd, int lds);
const void *stage_d3_f64(int n, int rd, int lds);
const void *stage_d4_f64(int n, int rd, int lds);
const void *stage_d5_f64(int n, int rd, int lds);
const void *stage_d6_f64(int n, int rd, int lds);
const void *stage_d2_f32(int n, int rd, int lds);
const void *stage_d3_f32(int n, int rd, int lds);
const void *stage_d4_f32(int n, int rd, int lds);
const void *stage_d5_f32(int n, int rd, int lds);
const void *stage_d6_f32(int n, int rd, int lds);

// Specialised kernel for d = 6 (3 x + 3 v), degree 3: one cell per
// 256-thread workgroup (stage_k3.hip); options as in hd_plan.
const void *stage_k3_f64(int options);
const void *stage_k3_f32(int options);

}  // namespace hd
