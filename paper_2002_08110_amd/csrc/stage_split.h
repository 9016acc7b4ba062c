// Dimension-split LSRK stage for cells too large to stage whole (d >= 5 at
// degree >= 4): the operator of stage_kernel.h evaluated in two passes.
//
// With collocation at the Gauss-Lobatto nodes the operator is a sum over
// dimensions of one-dimensional terms, and the term of dimension j at a node
// reads only the line of that node along j (plus one inflow trace value on
// the cell face), because a_j does not depend on x_j (Sec. 1.3; the strong
// form used by stage_kernel.h). In the canonical layout (dof = cell * n^d +
// node, node digits with dimension 1 fastest) the x-nodes of one velocity
// node tuple of a cell - a "row" of n^dx values - are contiguous, and the
// rows of a cell follow each other. So:
//
//   pass x: a workgroup stages R consecutive rows (of one or two cells) in
//           LDS and sums the x-dimension terms of each node: the sweeps along
//           the x dimensions and the inflow jumps from the rows of the
//           x-neighbour cells with the same velocity node tuple;
//   pass v: a workgroup stages C consecutive x-nodes of one cell in every row
//           (a "column block": all n^dv velocity node tuples) and adds the
//           velocity-dimension terms, whose lines run down the columns, with
//           the inflow jumps from the v-neighbour cells; then the RK update.
//
// A thread owns one line of n nodes (in pass x along x dimension 1, in pass
// v along the first velocity dimension): that sweep acts on its registers
// with coefficients common to the workgroup; the other sweeps read the n
// lines through the thread's nodes from LDS with the thread's row of the
// differentiation matrix; a line on an inflow face reads the neighbour's
// line from global memory.
//
// Between the passes the x-sum of every node waits in memory the stage would
// write anyway: in the output of an operator application; for an FP64 stage
// in the output solution vector (pass v reads it before overwriting it with
// the new solution at the same node, in the same thread); in FP32 operator
// mode folded into the increment (du <- A du + dt L_x in pass x, du <- du +
// dt L_v in pass v), whose FP32 width halves that round trip. A pass reads
// and writes only whole rows or column blocks, so a cell never has to fit
// on chip: traffic per DoF rises from the fused kernel's 32 B (FP64 middle
// stage) to 56 B, in exchange for small tiles at high occupancy.
//
// Dimensions contribute in the order 1..d, volume term then inflow jump, as
// in stage_kernel.h; results agree with it to rounding.
#pragma once

#include <type_traits>

#include "stage_kernel.h"

namespace hd {

// Tile shapes of the dimension-split passes for d dims, n = N nodes per
// dimension, dx configuration dimensions and operator values of PS bytes. A
// thread owns one line of N nodes: in pass x a line along x dimension 1 of
// one row, in pass v a line along the first velocity dimension of one column.
// Pass v takes as many columns as fit VT threads: 448 in FP64 (12 columns at
// degree 5, 7 waves) and 720 in FP32 operator mode (20 columns, 12 waves),
// the faster tile in each precision (at 6D degree 5: 2.38 ms per FP64 stage
// against 2.43 with 504 threads and 2.46 with 576; 1.71 ms per FP32 stage
// against 1.75 with 576 and 1.86 with 448).
template <int D, int N, int DX, int PS>
struct SplitShape {
  static constexpr int DV = D - DX;
  static constexpr int NXB = ipow(N, DX);  // nodes of a row (x-nodes of a cell)
  static constexpr int NVB = ipow(N, DV);  // rows of a cell
  static constexpr int ND = NXB * NVB;
  static constexpr int LX = ipow(N, DX - 1);  // lines of a row
  static constexpr int LV = ipow(N, DV - 1);  // lines of a column
  static constexpr int R = 256 / LX;          // rows per pass-x tile
  static constexpr int VT = PS == 4 ? 720 : 448;
  static constexpr int C = VT / LV < NXB ? VT / LV : NXB;  // columns per pass-v tile
  static constexpr int NCH = (NXB + C - 1) / C;  // column blocks per cell
  static constexpr int TX = (R * LX + 63) / 64 * 64;  // threads of pass x
  static constexpr int TV = (C * LV + 63) / 64 * 64;  // threads of pass v
  // LDS row stride of pass x (in values): two values of padding, so that
  // the lines read by the lanes of a wave spread over the banks. Pass v
  // stores its column block by velocity node tuple, a row of C values
  // (stride CS), so that the lanes of consecutive columns read consecutive
  // addresses.
  static constexpr int RS = NXB + 2;
  static constexpr int CS = C + 1;
  // LDS table Dm[N][N], read with per-lane row indices (a kernel argument
  // indexed at run time would be copied to scratch memory).
  static constexpr int NTAB = N * N;
  static_assert(R >= 1 && R <= NVB, "a pass-x tile spans at most two cells");
  static_assert(C >= 1 && C <= NXB, "a column block lies in one cell");
  static_assert(TX <= 1024 && TV <= 1024, "a workgroup holds at most 1024 threads");
};

// LDS of pass x: the table, the rows, the inflow-face lines of x dims 2..dx
// (per row and dim, the LX / N lines of the face); of pass v: the table, the
// column block, the face lines of velocity dims 2..dv (per dim, LV / N lines
// of N values, each by column).
template <int D, int N, int DX, typename P>
constexpr size_t split_x_lds_bytes() {
  using S = SplitShape<D, N, DX, sizeof(P)>;
  return (size_t)(S::NTAB + S::R * S::RS + S::R * (DX - 1) * S::LX) * sizeof(P);
}
template <int D, int N, int DX, typename P>
constexpr size_t split_v_lds_bytes() {
  using S = SplitShape<D, N, DX, sizeof(P)>;
  return (size_t)(S::NTAB + S::NVB * S::CS + (S::DV - 1) * S::LV * S::CS) * sizeof(P);
}

// q with base-N digit J removed (the index of a line on a face of dim J+1).
template <int N, int J>
__device__ __forceinline__ unsigned split_drop_digit(unsigned q) {
  constexpr unsigned st = (unsigned)ipow(N, J);
  return (q % st) + (q / (st * N)) * st;
}

// Multi-index of a cell (x dims first, dimension 1 fastest): one division
// per dimension, peeling the digits from the fastest.
template <int D, typename PV>
__device__ __forceinline__ void split_cell_index(PV &prm, unsigned cell, unsigned *c) {
  unsigned t = cell;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const unsigned q = j + 1 < D ? t / prm.cells[j] : 0u;
    c[j] = j + 1 < D ? t - q * prm.cells[j] : t;
    t = q;
  }
}

// Multi-index of cell + 1 from that of cell (digits carried; for the last
// cell the result wraps to cell 0, and no caller uses it then).
template <int D, typename PV>
__device__ __forceinline__ void split_next_index(PV &prm, const unsigned *c, unsigned *n) {
  bool carry = true;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const bool wrap = carry && c[j] + 1 == prm.cells[j];
    n[j] = carry ? (wrap ? 0u : c[j] + 1) : c[j];
    carry = wrap;
  }
}

// Periodic neighbour of `cell` (multi-index c) along dimension J: the left
// (c_J - 1) or the right one.
template <int J, typename PV>
__device__ __forceinline__ unsigned split_neighbour(PV &prm, unsigned cell, const unsigned *c, bool right) {
  const unsigned nj = prm.cells[J], st = prm.cstride[J];
  if (!right) return c[J] == 0 ? cell + (nj - 1) * st : cell - st;
  return c[J] == nj - 1 ? cell - (nj - 1) * st : cell + st;
}

// Base-N digit J of q, and q with that digit replaced by `dig`.
template <int N, int J>
__device__ __forceinline__ unsigned split_digit(unsigned q) {
  return (q / (unsigned)ipow(N, J)) % N;
}
template <int N, int J>
__device__ __forceinline__ unsigned split_set_digit(unsigned q, unsigned dig) {
  constexpr unsigned st = (unsigned)ipow(N, J);
  return q + (dig - split_digit<N, J>(q)) * st;
}

// The table Dm into LDS (one thread; compile-time indices), for reads after
// the workgroup's barrier.
template <int N, typename PV, typename P>
__device__ __forceinline__ void split_tables(PV &prm, P *tab) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N * N; ++q) tab[q] = prm.Dm[q];
  }
}

// Sweep along the thread's own line (uniform coefficients):
// sum[i] = sum_m Dm[i][m] v[m].
template <int N, typename PV, typename P>
__device__ __forceinline__ void split_own_sweep(PV &prm, const P *v, P *sum) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    P s = P(0);
#pragma unroll
    for (int m = 0; m < N; ++m) s += prm.Dm[i * N + m] * v[m];
    sum[i] = s;
  }
}

// Pass x: the x-dimension terms of R consecutive rows. Thread t owns the
// line along x dimension 1 with the other x digits l = t mod LX of row
// t / LX of the tile.
template <int D, int N, int DX, typename P, int OPT>
__global__ void __launch_bounds__((SplitShape<D, N, DX, sizeof(P)>::TX)) stage_split_x_kernel(const StageParams<P> prm) {
  using S = SplitShape<D, N, DX, sizeof(P)>;
  constexpr int NXB = S::NXB, NVB = S::NVB, R = S::R, LX = S::LX, RS = S::RS;
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr bool F32 = sizeof(P) == 4;
  extern __shared__ unsigned char smem_raw[];
  P *tab = reinterpret_cast<P *>(smem_raw);  // Dm
  P *lu = tab + S::NTAB;                     // [R][RS] the rows
  P *lf = lu + R * RS;                       // [R][DX-1][LX/N][N] face lines
  const unsigned tid = threadIdx.x;
  const unsigned tile = prm.xcd_remap ? xcd_tile(blockIdx.x, prm.nblocks) : blockIdx.x;
  const uint64_t nrows = (uint64_t)prm.ncells * NVB;
  const uint64_t g0 = (uint64_t)tile * R;
  if (g0 >= nrows) return;
  const unsigned nr = (unsigned)(nrows - g0 < (uint64_t)R ? nrows - g0 : (uint64_t)R);
  const bool stage = prm.mode == 1;
  split_tables<N>(prm, tab);

  const unsigned r = tid / LX, l = tid - r * LX;
  const bool active = r < nr;
  // The row's cell (the tile spans at most two) and velocity node tuple.
  const unsigned c0 = (unsigned)(g0 / NVB);
  const unsigned vt0 = (unsigned)(g0 - (uint64_t)c0 * NVB);
  const unsigned c1 = c0 + 1 < prm.ncells ? c0 + 1 : c0;
  unsigned ci0[D], ci1[D], ci[D];
  split_cell_index<D>(prm, c0, ci0);
  split_next_index<D>(prm, ci0, ci1);  // used only by rows of c1, which exist if c0 + 1 < ncells
  const bool cs = vt0 + r >= (unsigned)NVB;
  const unsigned vt = cs ? vt0 + r - NVB : vt0 + r;
  const unsigned cell = cs ? c1 : c0;
#pragma unroll
  for (int j = 0; j < D; ++j) ci[j] = cs ? ci1[j] : ci0[j];
  const uint64_t rbase = ((uint64_t)cell * NVB + vt) * NXB;
  const unsigned lbase = l * N;  // the line's first node in the row

  // Speeds a_j of the row: the constant, or v_{dx+j} at the row's velocity
  // node (phase-space field), formed as stage_kernel.h forms them.
  P a[DX];
  const bool phase = prm.field_kind == 1;
#pragma unroll
  for (int j = 0; j < DX; ++j) {
    if (!phase) {
      a[j] = prm.a_const[j];
    } else {
      const int m = DX + j < D ? DX + j : D - 1;
      const unsigned dig = (vt / (unsigned)ipow(N, j)) % N;
      // xi[dig] by a chain of selects over the kernel argument
      P xi = prm.xi[0];
#pragma unroll
      for (int q = 1; q < N; ++q) xi = dig == (unsigned)q ? prm.xi[q] : xi;
      a[j] = (prm.vlo[m] + P(ci[m]) * prm.vh[m]) + xi * prm.vh[m];
    }
  }

  // The line, the inflow traces and (FP32 stage) the increment.
  double u64[N] = {};
  double fx0 = 0.0;
  P dv[N];
  // Face line of x dim J (2..dx) of this thread's row, at the thread's
  // position in the face.
  auto face_at = [&](auto Jc) -> P * {
    constexpr int J = decltype(Jc)::value;
    return lf + ((r * (DX - 1) + (J - 1)) * (LX / N) + split_drop_digit<N, J - 1>(l)) * N;
  };
  // The loads go out together: the face lines into registers, to LDS once
  // every load has been issued (a store inside each face's branch would wait
  // for all earlier loads before the next face's loads could start).
  double fl[DX > 1 ? DX - 1 : 1][N];
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) u64[i] = prm.u_in[rbase + lbase + i];
    if (F32 && stage && prm.read_du) {
#pragma unroll
      for (int i = 0; i < N; ++i) dv[i] = ld_opt<NT>(prm.du + rbase + lbase + i);
    }
    // Dimension 1: one trace value at the line's inflow end.
    if (a[0] != P(0)) {
      const unsigned nb = cs ? split_neighbour<0>(prm, c1, ci1, a[0] < P(0))
                             : split_neighbour<0>(prm, c0, ci0, a[0] < P(0));
      const uint64_t nrow = ((uint64_t)nb * NVB + vt) * NXB;
      fx0 = prm.u_in[nrow + lbase + (a[0] > P(0) ? N - 1 : 0)];
    }
    // Dimensions 2..dx: the neighbour's line, if this one lies on the
    // inflow face.
    auto face = [&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      const unsigned ij = split_digit<N, J - 1>(l);
      const bool useL = ij == 0 && a[J] > P(0), useR = ij == N - 1 && a[J] < P(0);
      if (useL || useR) {
        const unsigned nb = cs ? split_neighbour<J>(prm, c1, ci1, useR)
                               : split_neighbour<J>(prm, c0, ci0, useR);
        const uint64_t nrow = ((uint64_t)nb * NVB + vt) * NXB;
        const unsigned nl = split_set_digit<N, J - 1>(l, useL ? N - 1 : 0);
#pragma unroll
        for (int i = 0; i < N; ++i) fl[J - 1][i] = prm.u_in[nrow + nl * N + i];
      }
    };
    if constexpr (DX > 1) face(std::integral_constant<int, 1>{});
    if constexpr (DX > 2) face(std::integral_constant<int, 2>{});
    // FP32: the empty asm keeps the conversions out of the load branches
    // (the compiler would convert right after each load, and wait for it,
    // before the next face's loads).
    if constexpr (F32) {
      asm volatile("" : "+v"(fx0));
#pragma unroll
      for (int j = 0; j < (DX > 1 ? DX - 1 : 1); ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) asm volatile("" : "+v"(fl[j][i]));
    }
#pragma unroll
    for (int i = 0; i < N; ++i) lu[r * RS + lbase + i] = to_p<P>(u64[i]);
    auto face_store = [&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      const unsigned ij = split_digit<N, J - 1>(l);
      if ((ij == 0 && a[J] > P(0)) || (ij == N - 1 && a[J] < P(0))) {
        P *f = face_at(Jc);
#pragma unroll
        for (int i = 0; i < N; ++i) f[i] = to_p<P>(fl[J - 1][i]);
      }
    };
    if constexpr (DX > 1) face_store(std::integral_constant<int, 1>{});
    if constexpr (DX > 2) face_store(std::integral_constant<int, 2>{});
  }
  __syncthreads();

  P up[N], acc[N], sum[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    up[i] = to_p<P>(u64[i]);
    acc[i] = P(0);
  }
  if (active) {
  // Dimension 1 on the thread's registers.
  split_own_sweep<N>(prm, up, sum);
  {
    const P c = a[0] * prm.inv_h[0];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] -= c * sum[i];
    const P lf0 = prm.lift_inv_h[0];
    const P f0 = to_p<P>(fx0);
    if (a[0] > P(0)) acc[0] += lf0 * a[0] * (f0 - up[0]);
    if (a[0] < P(0)) acc[N - 1] += -lf0 * a[0] * (f0 - up[N - 1]);
  }
  // Dimensions 2..dx: the lines through the thread's nodes from LDS, with
  // the thread's row of Dm.
  auto sweep = [&](auto Jc) {
    constexpr int J = decltype(Jc)::value;
    const unsigned ij = split_digit<N, J - 1>(l);
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = tab[ij * N + m];
#pragma unroll
    for (int i = 0; i < N; ++i) sum[i] = P(0);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const unsigned lm = split_set_digit<N, J - 1>(l, m);
#pragma unroll
      for (int i = 0; i < N; ++i) sum[i] += row[m] * lu[r * RS + lm * N + i];
    }
    const P c = a[J] * prm.inv_h[J];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] -= c * sum[i];
    const bool useL = ij == 0 && a[J] > P(0), useR = ij == N - 1 && a[J] < P(0);
    if (useL || useR) {
      const P lfj = prm.lift_inv_h[J];
      const P w = useL ? lfj * a[J] : -lfj * a[J];
      const P *f = face_at(Jc);
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] += w * (f[i] - up[i]);
    }
  };
  if constexpr (DX > 1) sweep(std::integral_constant<int, 1>{});
  if constexpr (DX > 2) sweep(std::integral_constant<int, 2>{});
  // The result: the x-sum, or (FP32 stage) the increment with A du folded in.
  if constexpr (F32) {
    if (stage) {
#pragma unroll
      for (int i = 0; i < N; ++i)
        acc[i] = prm.read_du ? rk_fma(prm.rk_a, dv[i], prm.dt * acc[i]) : prm.dt * acc[i];
    }
  }
  }  // active

  // Out through the LDS rows (once every thread has read them for its
  // sweeps): the tile's rows are contiguous in memory, and consecutive lanes
  // then store consecutive values (a thread's own line would leave every
  // 64-byte sector to three partial stores).
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) lu[r * RS + lbase + i] = acc[i];
  }
  __syncthreads();
  const uint64_t base = g0 * NXB;
  const unsigned tn = nr * NXB;
  for (unsigned n = tid; n < tn; n += S::TX) {
    const unsigned rr = n / NXB, x = n - rr * NXB;
    const P v = lu[rr * RS + x];
    if (!stage) prm.out[base + n] = v;
    else if constexpr (F32) st_opt<NT>(prm.du + base + n, v);
    else st_opt<NT>(prm.u_out + base + n, (double)v);
  }
}

// Pass v: the velocity-dimension terms of C x-nodes in every row of one
// cell, added to the x-sum of pass x, and the RK update. Thread t owns the
// line along the first velocity dimension of column x0 + t mod C with the
// other velocity digits q = t / C.
template <int D, int N, int DX, typename P, int OPT>
__global__ void __launch_bounds__((SplitShape<D, N, DX, sizeof(P)>::TV)) stage_split_v_kernel(const StageParams<P> prm) {
  using S = SplitShape<D, N, DX, sizeof(P)>;
  constexpr int DV = S::DV, NXB = S::NXB, C = S::C, LV = S::LV, NCH = S::NCH, CS = S::CS;
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr bool F32 = sizeof(P) == 4;
  extern __shared__ unsigned char smem_raw[];
  P *tab = reinterpret_cast<P *>(smem_raw);  // Dm
  P *lc = tab + S::NTAB;                     // [NVB][CS] the column block
  P *lf = lc + S::NVB * CS;                  // [DV-1][LV/N][N][CS] face lines
  const unsigned tid = threadIdx.x;
  const unsigned tile = prm.xcd_remap ? xcd_tile(blockIdx.x, prm.nblocks) : blockIdx.x;
  const unsigned cell = tile / NCH;
  if (cell >= prm.ncells) return;
  const unsigned x0 = (tile - cell * NCH) * C;
  const unsigned cw = NXB - x0 < (unsigned)C ? NXB - x0 : (unsigned)C;
  const bool stage = prm.mode == 1;
  split_tables<N>(prm, tab);

  const unsigned q = tid / C, xc = tid - q * C;
  const bool active = q < (unsigned)LV && xc < cw;
  unsigned ci[D];
  split_cell_index<D>(prm, cell, ci);
  unsigned xcell = 0;
#pragma unroll
  for (int m = 0; m < DX; ++m) xcell += ci[m] * prm.cstride[m];
  const uint64_t cbase = (uint64_t)cell * S::ND + x0 + xc;  // the column's node 0
  // Node i of the thread's line: velocity node tuple i + N q.
  auto at = [&](unsigned qq, int i) -> uint64_t { return cbase + (uint64_t)(i + N * qq) * NXB; };

  // Node i of the face line of velocity dim JJ (2..dv) at this thread's
  // position in the face.
  auto face_at = [&](auto Jc, int i) -> P & {
    constexpr int JJ = decltype(Jc)::value;
    return lf[(((JJ - 1) * (LV / N) + split_drop_digit<N, JJ - 1>(q)) * N + i) * CS + xc];
  };
  // The loads are written without branches inside unrolled loops (uniform
  // choices select a pointer) so that they form one block: every load that
  // does not depend on the field is in flight while the field arrives, and
  // the inflow-face loads that do depend on it go out together.
  P a[DV];
  const bool phase = prm.field_kind == 1;
  double u64[N];
  double fv0 = 0.0;
  P part[N], dv[N];
  double fl[DV > 1 ? DV - 1 : 1][N];
  if (active) {
    // FP64 stage increment (stages after the first): its own uniform branch,
    // ahead of the rest.
    if constexpr (!F32) {
#pragma unroll
      for (int i = 0; i < N; ++i) dv[i] = P(0);
      if (stage && prm.read_du) {
#pragma unroll
        for (int i = 0; i < N; ++i) dv[i] = ld_opt<NT>(prm.du + at(q, i));
      }
    }
    // Speeds of the velocity dims at the column's x-node: esign E
    // (phase-space field) or the constants. Without the field the load reads
    // the solution's first value, a valid address, and is discarded.
    const P *eb = phase ? prm.E + ((uint64_t)xcell * NXB + x0 + xc) * DX
                        : reinterpret_cast<const P *>(prm.u_in);
    P er[DV];
#pragma unroll
    for (int jj = 0; jj < DV; ++jj) er[jj] = eb[phase ? jj : 0];
#pragma unroll
    for (int i = 0; i < N; ++i) u64[i] = prm.u_in[at(q, i)];
    // The x-sum (FP64 stage: the output solution; operator application: the
    // output) or, in FP32 operator mode, the increment that holds it.
    {
      const P *ps;
      if constexpr (F32) ps = stage ? prm.du : prm.out;
      else ps = stage ? reinterpret_cast<const P *>(prm.u_out) : prm.out;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const P v = ld_opt<NT>(ps + at(q, i));
        if constexpr (F32) {
          part[i] = stage ? P(0) : v;
          dv[i] = stage ? v : P(0);
        } else {
          part[i] = v;
        }
      }
    }
    // The field values are first used here, behind the loads above: the
    // empty asm keeps the compiler from moving their loads into the branch
    // of the phase-space field, where each would wait for all the others.
#pragma unroll
    for (int jj = 0; jj < DV; ++jj) asm volatile("" : "+v"(er[jj]));
#pragma unroll
    for (int jj = 0; jj < DV; ++jj) a[jj] = phase ? prm.esign * er[jj] : prm.a_const[DX + jj];
    // First velocity dim: one trace value at the line's inflow end.
    if (a[0] != P(0)) {
      const unsigned nb = split_neighbour<DX>(prm, cell, ci, a[0] < P(0));
      const uint64_t nbase = (uint64_t)nb * S::ND + x0 + xc;
      fv0 = prm.u_in[nbase + (uint64_t)((a[0] > P(0) ? N - 1 : 0) + N * q) * NXB];
    }
    // Velocity dims 2..dv: the neighbour's line, if this one lies on the
    // inflow face, into registers (to LDS below, once every load is out).
    auto face = [&](auto Jc) {
      constexpr int JJ = decltype(Jc)::value;
      const unsigned ij = split_digit<N, JJ - 1>(q);
      const bool useL = ij == 0 && a[JJ] > P(0), useR = ij == N - 1 && a[JJ] < P(0);
      if (useL || useR) {
        const unsigned nb = split_neighbour<DX + JJ>(prm, cell, ci, useR);
        const uint64_t nbase = (uint64_t)nb * S::ND + x0 + xc;
        const unsigned nq = split_set_digit<N, JJ - 1>(q, useL ? N - 1 : 0);
#pragma unroll
        for (int i = 0; i < N; ++i) fl[JJ - 1][i] = prm.u_in[nbase + (uint64_t)(i + N * nq) * NXB];
      }
    };
    if constexpr (DV > 1) face(std::integral_constant<int, 1>{});
    if constexpr (DV > 2) face(std::integral_constant<int, 2>{});
    if constexpr (F32) {
      asm volatile("" : "+v"(fv0));
#pragma unroll
      for (int j = 0; j < (DV > 1 ? DV - 1 : 1); ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) asm volatile("" : "+v"(fl[j][i]));
    }
#pragma unroll
    for (int i = 0; i < N; ++i) lc[(N * q + i) * CS + xc] = to_p<P>(u64[i]);
    auto face_store = [&](auto Jc) {
      constexpr int JJ = decltype(Jc)::value;
      const unsigned ij = split_digit<N, JJ - 1>(q);
      if ((ij == 0 && a[JJ] > P(0)) || (ij == N - 1 && a[JJ] < P(0))) {
#pragma unroll
        for (int i = 0; i < N; ++i) face_at(Jc, i) = to_p<P>(fl[JJ - 1][i]);
      }
    };
    if constexpr (DV > 1) face_store(std::integral_constant<int, 1>{});
    if constexpr (DV > 2) face_store(std::integral_constant<int, 2>{});
  }
  __syncthreads();
  if (!active) return;

  P up[N], acc[N], sum[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    up[i] = to_p<P>(u64[i]);
    acc[i] = F32 && stage ? P(0) : part[i];
  }
  // First velocity dim on the thread's registers.
  split_own_sweep<N>(prm, up, sum);
  {
    const P c = a[0] * prm.inv_h[DX];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] -= c * sum[i];
    const P lf0 = prm.lift_inv_h[DX];
    const P f0 = to_p<P>(fv0);
    if (a[0] > P(0)) acc[0] += lf0 * a[0] * (f0 - up[0]);
    if (a[0] < P(0)) acc[N - 1] += -lf0 * a[0] * (f0 - up[N - 1]);
  }
  auto sweep = [&](auto Jc) {
    constexpr int JJ = decltype(Jc)::value;
    const unsigned ij = split_digit<N, JJ - 1>(q);
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = tab[ij * N + m];
#pragma unroll
    for (int i = 0; i < N; ++i) sum[i] = P(0);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const unsigned qm = split_set_digit<N, JJ - 1>(q, m);
#pragma unroll
      for (int i = 0; i < N; ++i) sum[i] += row[m] * lc[(N * qm + i) * CS + xc];
    }
    const P c = a[JJ] * prm.inv_h[DX + JJ];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] -= c * sum[i];
    const bool useL = ij == 0 && a[JJ] > P(0), useR = ij == N - 1 && a[JJ] < P(0);
    if (useL || useR) {
      const P lfj = prm.lift_inv_h[DX + JJ];
      const P w = useL ? lfj * a[JJ] : -lfj * a[JJ];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] += w * (face_at(Jc, i) - up[i]);
    }
  };
  if constexpr (DV > 1) sweep(std::integral_constant<int, 1>{});
  if constexpr (DV > 2) sweep(std::integral_constant<int, 2>{});

  if (!stage) {
#pragma unroll
    for (int i = 0; i < N; ++i) prm.out[at(q, i)] = acc[i];
    return;
  }
  P d[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if constexpr (F32) d[i] = rk_fma(prm.dt, acc[i], dv[i]);
    else d[i] = prm.read_du ? rk_fma(prm.rk_a, dv[i], prm.dt * acc[i]) : prm.dt * acc[i];
  }
  if (prm.write_du) {
#pragma unroll
    for (int i = 0; i < N; ++i) st_opt<NT>(prm.du + at(q, i), d[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) st_opt<NT>(prm.u_out + at(q, i), rk_fma(prm.rk_b, (double)d[i], u64[i]));
}

}  // namespace hd
