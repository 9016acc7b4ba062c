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
template <int D, int N, int DX, typename P>
constexpr bool gauss_compiled() {
  return (size_t)gauss_lds_elems(D, N, DX) * sizeof(P) + 1024 <= kMaxLdsBytes;
}

template <int D, int N, int DX, typename P>
const void *gauss_fn() {
  if constexpr (gauss_compiled<D, N, DX, P>())
    return reinterpret_cast<const void *>(&stage_gauss_kernel<D, N, DX, P>);
  else
    return nullptr;
}

template <int D, int DX, typename P>
const void *gauss_by_n(int n) {
  switch (n) {
    case 2: return gauss_fn<D, 2, DX, P>();
    case 3: return gauss_fn<D, 3, DX, P>();
    case 4: return gauss_fn<D, 4, DX, P>();
    case 5: return gauss_fn<D, 5, DX, P>();
    case 6: return gauss_fn<D, 6, DX, P>();
  }
  return nullptr;
}

template <typename P>
const void *gauss_by_d(int d, int n) {
  switch (d) {
    case 2: return gauss_by_n<2, 1, P>(n);
    case 3: return gauss_by_n<3, 2, P>(n);
    case 4: return gauss_by_n<4, 2, P>(n);
    case 5: return gauss_by_n<5, 3, P>(n);
    case 6: return gauss_by_n<6, 3, P>(n);
  }
  return nullptr;
}

}  // namespace

const void *stage_gauss_entry(int d, int n, bool f32) {
  return f32 ? gauss_by_d<float>(d, n) : gauss_by_d<double>(d, n);
}

}  // namespace hd
