// Entries of the dimension-split stage passes (stage_split.h): d = 6 (3 x +
// 3 v) and d = 5 (3 + 2) at degrees 4 and 5.
#include "stage_dispatch.h"
#include "stage_split.h"

namespace hd {

namespace {

template <int D, int N, int DX, typename P, int OPT>
SplitEntry split_entry_of() {
  SplitEntry e;
  e.fx = reinterpret_cast<const void *>(&stage_split_x_kernel<D, N, DX, P, OPT>);
  e.fv = reinterpret_cast<const void *>(&stage_split_v_kernel<D, N, DX, P, OPT>);
  using S = SplitShape<D, N, DX, sizeof(P)>;
  static_assert(split_x_lds_bytes<D, N, DX, P>() <= kMaxLdsBytes &&
                    split_v_lds_bytes<D, N, DX, P>() <= kMaxLdsBytes,
                "the tiles of both passes fit the LDS of a workgroup");
  e.rows_per_tile = S::R;
  e.cols_per_tile = S::C;
  e.tiles_per_cell = S::NCH;
  e.threads_x = S::TX;
  e.threads_v = S::TV;
  e.lds_x = split_x_lds_bytes<D, N, DX, P>();
  e.lds_v = split_v_lds_bytes<D, N, DX, P>();
  return e;
}

template <int D, int N, int DX, typename P>
SplitEntry split_entry_opt(int options) {
  return (options & kOptStream) ? split_entry_of<D, N, DX, P, kOptStream>()
                                : split_entry_of<D, N, DX, P, 0>();
}

template <int D, int DX, typename P>
SplitEntry split_entry_n(int n, int options) {
  switch (n) {
    case 5: return split_entry_opt<D, 5, DX, P>(options);
    case 6: return split_entry_opt<D, 6, DX, P>(options);
  }
  return SplitEntry{};
}

template <typename P>
SplitEntry split_entry_p(int d, int dx, int n, int options) {
  if (d == 6 && dx == 3) return split_entry_n<6, 3, P>(n, options);
  if (d == 5 && dx == 3) return split_entry_n<5, 3, P>(n, options);
  return SplitEntry{};
}

}  // namespace

SplitEntry stage_split_entry(int d, int dx, int n, bool f32, int options) {
  return f32 ? split_entry_p<float>(d, dx, n, options) : split_entry_p<double>(d, dx, n, options);
}

}  // namespace hd
