// Entries of the Gauss-Legendre stage kernel: d = 2..6 (x/v split as for the
// collocation kernels), degree 1..5, FP64 and FP32; only variants whose LDS
// (U and the accumulated operator, one face layer, E at the x-Gauss points,
// the 1D tables) fits 160 KiB exist.
#include "stage_dispatch.h"
#include "stage_gauss.h"

namespace hd {
namespace {

// 1 KiB is kept free for the kernel's static LDS (the workgroup reduction
// behind __syncthreads_or).
// The mapped 5D degree-5 variant is left out: hipcc for gfx950 rejects it
// with an instruction-selection error.
template <int D, int N, int DX, typename P, bool M>
constexpr bool gauss_compiled() {
  return (size_t)gauss_lds_elems(D, N, DX, M, (int)sizeof(P)) * sizeof(P) + 1024 <= kMaxLdsBytes &&
         !(M && D == 5 && N == 6);
}

template <int D, int N, int DX, typename P, bool M>
const void *gauss_fn() {
  if constexpr (gauss_compiled<D, N, DX, P, M>())
    return reinterpret_cast<const void *>(&stage_gauss_kernel<D, N, DX, P, M>);
  else
    return nullptr;
}

template <int D, int DX, typename P, bool M>
const void *gauss_by_n(int n) {
  switch (n) {
    case 2: return gauss_fn<D, 2, DX, P, M>();
    case 3: return gauss_fn<D, 3, DX, P, M>();
    case 4: return gauss_fn<D, 4, DX, P, M>();
    case 5: return gauss_fn<D, 5, DX, P, M>();
    case 6: return gauss_fn<D, 6, DX, P, M>();
  }
  return nullptr;
}

template <typename P, bool M>
const void *gauss_by_d(int d, int n) {
  switch (d) {
    case 2: return gauss_by_n<2, 1, P, M>(n);
    case 3: return gauss_by_n<3, 2, P, M>(n);
    case 4: return gauss_by_n<4, 2, P, M>(n);
    case 5: return gauss_by_n<5, 3, P, M>(n);
    case 6: return gauss_by_n<6, 3, P, M>(n);
  }
  return nullptr;
}

}  // namespace

const void *stage_gauss_entry(int d, int n, bool f32, bool mapped) {
  if (mapped) return f32 ? gauss_by_d<float, true>(d, n) : gauss_by_d<double, true>(d, n);
  return f32 ? gauss_by_d<float, false>(d, n) : gauss_by_d<double, false>(d, n);
}

}  // namespace hd
