// Kernel resolution for the fused stage: from runtime (d, degree, register
// dims, LDS mode, precision) to the entry of the compiled variant. Each
// stage_dN.hip translation unit instantiates the kernels of one dimension d
// (all degrees, both precisions, both LDS modes, the valid register-dim
// counts) so the instantiations compile in parallel. The caller launches the
// returned entry with hipLaunchKernel (after raising its dynamic-LDS limit
// when a launch needs more than 64 KiB). Resolution makes no HIP call.
#pragma once

#include "stage_kernel.h"

namespace hd {

constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

struct LaunchShape {
  unsigned grid, block;
  size_t shmem;
};


// True if the LDS variant of (D, N, RD, P) can hold at least one cell.
template <int D, int N, int RD, typename P>
constexpr bool lds_variant_ok() {
  return ipow(N, D - RD) <= 1024 && (size_t)ipow(N, D) * sizeof(P) <= kMaxLdsBytes;
}

// True if the slab variant (SD split dims) of (D, N, RD, P) is compiled: it
// serves the cells that do not fit LDS whole (degree >= 4, d >= 5), and a
// slab must fit one workgroup and its LDS.
template <int D, int N, int DX, int RD, int SD, typename P>
constexpr bool split_variant_ok() {
  return SD >= 1 && N >= 5 && D >= 5 && RD + SD <= D - DX && D - RD - SD >= DX &&
         ipow(N, D - RD - SD) <= 1024 &&
         (size_t)ipow(N, D - SD) * sizeof(P) <= kMaxLdsBytes;
}

// True if the looped variant (a thread covers the N pencils of the slowest
// fast dimension) of (D, N, RD, SD, P) is compiled: units of more than 1024
// pencils at degree >= 4, d >= 5, that fit LDS; the looped dimension is a
// velocity dimension.
template <int D, int N, int DX, int RD, int SD, typename P>
constexpr bool loop_variant_ok() {
  return N >= 5 && D >= 5 && RD + SD <= D - DX && D - RD - SD >= DX + 1 &&
         ipow(N, D - RD - SD - 1) <= 1024 &&
         (size_t)ipow(N, D - SD) * sizeof(P) <= kMaxLdsBytes;
}

// list != 0: the persistent work-list form of the same variant
// (stage_list_kernel), which takes a ListParams<P> argument.
template <int D, int N, int DX, int RD, typename P, bool LDS, int SD, int OPT, int LD>
const void *variant_fn(int list) {
  if (list) return reinterpret_cast<const void *>(&stage_list_kernel<D, N, DX, RD, P, LDS, SD, OPT, LD>);
  return reinterpret_cast<const void *>(&stage_kernel<D, N, DX, RD, P, LDS, SD, OPT, LD>);
}

template <int D, int N, int DX, int RD, typename P, bool LDS, int SD, int LD = 0>
const void *resolve_opt(int opt, int list) {
  return (opt & kOptStream) ? variant_fn<D, N, DX, RD, P, LDS, SD, kOptStream, LD>(list)
                            : variant_fn<D, N, DX, RD, P, LDS, SD, 0, LD>(list);
}

template <int D, int N, int DX, int RD, typename P, int SD>
const void *resolve_loop(int lds, int opt, int list) {
  if constexpr (loop_variant_ok<D, N, DX, RD, SD, P>())
    return lds ? resolve_opt<D, N, DX, RD, P, true, SD, 1>(opt, list) : nullptr;
  return nullptr;
}

template <int D, int N, int DX, int RD, typename P>
const void *resolve_lds(int lds, int sd, int opt, int ld, int list) {
  if (ld == 1) {
    if (sd == 0) return resolve_loop<D, N, DX, RD, P, 0>(lds, opt, list);
    if (sd == 1) return resolve_loop<D, N, DX, RD, P, 1>(lds, opt, list);
    if (sd == 2) return resolve_loop<D, N, DX, RD, P, 2>(lds, opt, list);
    return nullptr;
  }
  if (ld != 0) return nullptr;
  if (sd == 1) {
    if constexpr (split_variant_ok<D, N, DX, RD, 1, P>())
      return lds ? resolve_opt<D, N, DX, RD, P, true, 1>(opt, list) : nullptr;
    return nullptr;
  }
  if (sd == 2) {
    if constexpr (split_variant_ok<D, N, DX, RD, 2, P>())
      return lds ? resolve_opt<D, N, DX, RD, P, true, 2>(opt, list) : nullptr;
    return nullptr;
  }
  if (sd != 0) return nullptr;
  if (lds) {
    if constexpr (lds_variant_ok<D, N, RD, P>()) return resolve_opt<D, N, DX, RD, P, true, 0>(opt, list);
    else return nullptr;
  }
  return resolve_opt<D, N, DX, RD, P, false, 0>(opt, list);
}

template <int D, int N, int DX, typename P>
const void *resolve_rd(int rd, int lds, int sd, int opt, int ld, int list) {
  constexpr int DV = D - DX;
  if (rd == 1) return resolve_lds<D, N, DX, 1, P>(lds, sd, opt, ld, list);
  if constexpr (DV >= 2) {
    if (rd == 2) return resolve_lds<D, N, DX, 2, P>(lds, sd, opt, ld, list);
  }
  return nullptr;
}

template <int D, int DX, typename P>
const void *resolve_n(int n, int rd, int lds, int sd, int opt, int ld, int list) {
  switch (n) {
    case 2: return resolve_rd<D, 2, DX, P>(rd, lds, sd, opt, ld, list);
    case 3: return resolve_rd<D, 3, DX, P>(rd, lds, sd, opt, ld, list);
    case 4: return resolve_rd<D, 4, DX, P>(rd, lds, sd, opt, ld, list);
    case 5: return resolve_rd<D, 5, DX, P>(rd, lds, sd, opt, ld, list);
    case 6: return resolve_rd<D, 6, DX, P>(rd, lds, sd, opt, ld, list);
    default: return nullptr;
  }
}

// Defined in stage_dN_fP.hip (one per dimension and precision): the entry of
// the generic kernel for n = degree + 1 nodes per dimension, rd register
// dims, LDS mode, sd split dims, plan options opt and ld looped dims (list:
// its persistent work-list form), or nullptr if that variant is not
// compiled.
const void *stage_d2_f64(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d3_f64(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d4_f64(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d5_f64(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d6_f64(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d2_f32(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d3_f32(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d4_f32(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d5_f32(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);
const void *stage_d6_f32(int n, int rd, int lds, int sd, int opt, int ld, int list = 0);

// Specialised kernel for d = 6 (3 x + 3 v), degree 3: one cell per
// 256-thread workgroup (stage_k3.hip); options as in hd_plan.
// role: 0 general (operator application, any stage), 1 first stage
// (read_du == 0), 2 late increment (any stage after the first)
// list != 0: the persistent work-list form (stage_k3_list_kernel).
const void *stage_k3_f64(int options, int role = 0, int list = 0);
const void *stage_k3_f32(int options, int role = 0, int list = 0);

// Gauss-Legendre quadrature for d = 6 (3 x + 3 v), degree 3, Cartesian
// cells, in the thread layout of the collocation kernel above
// (stage_k3_gauss.hip); streaming stores.
const void *stage_k3g_entry(bool f32);

// Gauss-Lobatto collocation on mapped cells for d = 6 (3 x + 3 v), degree
// 3, in the same layout (stage_k3_mapped.hip); streaming stores.
const void *stage_k3m_entry(bool f32);

// Gauss-Legendre quadrature on mapped cells for d = 6 (3 x + 3 v), degree 3,
// in the same layout (stage_k3_mgauss.hip); streaming stores.
const void *stage_k3mg_entry(bool f32);

// Sweep kernel (stage_gauss.hip): Gauss-Legendre quadrature on Cartesian
// cells, or either quadrature on mapped cells; one cell per workgroup;
// nullptr where the cell's LDS does not fit.
const void *stage_gauss_entry(int d, int n, bool f32, bool mapped = false);

// Dimension-split passes (stage_split.hip): pass x over tiles of
// rows_per_tile consecutive rows (the n^dx x-nodes of one velocity node
// tuple of a cell), threads_x threads and lds_x bytes of LDS; pass v over
// tiles_per_cell column blocks of each cell (cols_per_tile x-nodes in every
// row), threads_v threads and lds_v bytes. Compiled for d = 6 (3 + 3) and d = 5
// (3 + 2) at degrees 4 and 5 with Gauss-Lobatto collocation on Cartesian
// cells; null entries otherwise. options as in hd_plan (bit 0).
struct SplitEntry {
  const void *fx = nullptr, *fv = nullptr;
  int rows_per_tile = 0, cols_per_tile = 0, tiles_per_cell = 0;
  unsigned threads_x = 0, threads_v = 0;
  size_t lds_x = 0, lds_v = 0;
};
SplitEntry stage_split_entry(int d, int dx, int n, bool f32, int options);

}  // namespace hd
