// Fused element-centric DG advection stage kernel for gfx950.
//
// One thread owns a "pencil": the (k+1)^RD nodes of one cell that share the
// thread's index in the NF fastest node dimensions. Derivatives along the RD
// slowest dimensions act on the thread's own registers; derivatives along
// the NF fast dimensions read the other nodes of the line from LDS (the
// cell is staged there once) or from global memory. Cells too large for LDS
// can be cut into slabs along SD "split" dimensions (velocity dimensions
// between the fast and the register ones): a workgroup then stages one slab,
// the nodes with one fixed digit tuple in the split dimensions, and the
// derivatives along a split dimension read the other slabs of the cell from
// global memory (cache hits: the slabs of a cell run on neighbouring
// workgroups). Every output value is written by exactly one thread and the
// input vector is read-only, so the element-centric loop is race free
// (Sec. 2.6).
//
// Per node i of cell c the kernel evaluates, for each dimension j,
//   -a_j/h_j * sum_m D[i_j][m] u_{i_j->m}                    (volume)
//   + lift/h_j * max(a_j,0) * (u^-_{c-e_j} - u_i)  if i_j = 0   (inflow face)
//   - lift/h_j * min(a_j,0) * (u^+_{c+e_j} - u_i)  if i_j = k   (inflow face)
// with D[q][m] = l'_m(xi_q) and lift = 1/w_0 = 1/w_k. This is the strong
// form of the collocated weak form of Sec. 1.3 / Algorithm 2: for
// Gauss-Lobatto collocation the summation-by-parts identity
// W D + D^T W = diag(-1, 0, .., 0, 1) turns the weak volume term plus the
// outflow (own-trace) face terms into -a D u, leaving only the jump on the
// inflow face. The inverse mass matrix is diagonal (collocation) and is
// folded into the coefficients. a_j never depends on x_j for the supported
// fields (constant; a_x = v, a_v = E(x)), so a_j factors out of the line sum.
// The dimensions contribute in the order j = 1..d (volume, then face) in
// every variant.
//
// The low-storage RK update (Sec. 5.4) is fused into the same pass:
//   du <- A_s du + dt L(u),  u_out <- u_in + B_s du.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "work_list.h"

namespace hd {

constexpr int kMaxN = 6;   // degree <= 5
constexpr int kMaxD = 6;

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Kernel parameters, typed on the operator precision P.
template <typename P>
struct StageParams {
  const double *u_in;   // FP64 solution in
  double *u_out;        // FP64 solution out (stage mode)
  P *du;                // stage increment (read if read_du, written if write_du)
  P *out;               // operator output (apply mode)
  const P *E;           // E at x-nodes: [(xcell * n^dx + xnode) * dx + comp]
  unsigned ncells;
  unsigned nblocks;     // blocks launched (for the XCD remap)
  unsigned cells_per_wg;
  unsigned cells[kMaxD];
  unsigned cstride[kMaxD];
  int mode;             // 0: out = L(u_in); 1: fused RK stage
  int read_du, write_du;
  int field_kind;       // 0: constant; 1: phase space
  int xcd_remap;
  double rk_b;          // B_s (FP64: applied to the FP64 solution)
  P rk_a;               // A_s
  P dt;
  P inv_h[kMaxD];
  P lift_inv_h[kMaxD];  // lift / h_j
  P a_const[kMaxD];
  P vlo[kMaxD], vh[kMaxD];  // node coordinate lo_j + (c_j + xi_i) h_j
  P xi[kMaxN];
  P Dm[kMaxN * kMaxN];  // Dm[q * N + m] = l'_m(xi_q) on [0, 1]
  P esign;
  // Stage mode of the 6D degree-3 kernel under the Vlasov-Poisson field:
  // per thread, the velocity moment of its 16 output values over (i5, i6),
  // sum_i6 gw[i6] sum_i5 gw[i5] u_out, at vp_mom[cell * 256 + thread]; null
  // otherwise.
  double *vp_mom;
  double gw[kMaxN];     // Gauss-Lobatto weights on [0, 1]
  // Mapped configuration cells: per x-cell, the metric at the quadrature
  // points (layout in stage_gauss.h); null for Cartesian cells.
  const double *xmetric;
};

// Map the hardware workgroup id (dispatched round-robin over the 8 XCDs) to a
// tile index so that each XCD processes one contiguous range of tiles; the
// face neighbours along the fast cell dimensions then share that XCD's L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblocks) {
  const unsigned x = b & 7u, idx = b >> 3;
  const unsigned q = nblocks >> 3, r = nblocks & 7u;
  return x * q + (x < r ? x : r) + idx;
}

// Scheduling fence: keeps the compiler from hoisting the loads of later
// dimensions above this point, which would multiply live registers.
// (An empty asm statement with a memory clobber: memory operations are not
// moved across it, at the IR or the machine level.)
__device__ __forceinline__ void sched_fence() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");
}

// Pin a value in a register at this point of the program: the computation
// producing it cannot be sunk below (an empty asm that reads and writes it).
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(float &x) { asm volatile("" : "+v"(x)); }

template <typename P>
__device__ __forceinline__ P to_p(double v) {
  return static_cast<P>(v);
}

// The low-storage RK update with one fixed rounding order: the increment
// du' = fma(A_s, du, dt L) (dt L rounded first) and u' = fma(B_s, du', u).
// Written out, a*b + c*d may be fused either way round, and two kernels
// compiled from the same source (a solve's own launch and its batched
// work-list form) could round differently.
__device__ __forceinline__ float rk_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double rk_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Plan option bit 0: non-temporal (streaming) loads and stores of the stage
// increment and stores of the output solution, which are not re-read while
// they could still be cached; keeps the cache for neighbour traces.
constexpr int kOptStream = 1;

template <bool NT, typename T>
__device__ __forceinline__ T ld_opt(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_opt(T *p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Largest workgroup a variant is launched with: 256 threads, except the LDS
// variant of units (cells or slabs) with more than 256 pencils, which takes
// one unit per workgroup (its pencil count, rounded up to whole waves).
template <int D, int N, int RD, bool USE_LDS, int SD, int LD = 0>
constexpr int stage_max_threads() {
  constexpr int T = ipow(N, D - RD - SD - LD);
  return (USE_LDS && T > 256) ? (T + 63) / 64 * 64 : 256;
}

// One workgroup's share of a stage: the tile `tile` (cells_per_wg units -
// cells, or slabs of cells if SD > 0 - for the LDS variant; blockDim.x
// pencils otherwise). lds_reuse: the LDS of a previous tile may still be
// read by other threads, so wait before overwriting it. OPT: plan options.
// LD = 1 (LDS variant): a thread covers the N pencils that differ in the
// slowest fast dimension one after another, so a unit of N^NF pencils runs
// on N^(NF-1) threads: large units fit a workgroup, and the sweep along that
// dimension still reads LDS.
template <int D, int N, int DX, int RD, typename P, bool USE_LDS, int SD, int OPT, int LD = 0,
          typename PV = const StageParams<P>>
__device__ __forceinline__ void stage_body(PV &prm, unsigned tile, P *lds, bool lds_reuse,
                                           const unsigned tid) {
  constexpr int DV = D - DX;
  static_assert(RD >= 1 && RD + SD <= DV, "register and split dims must be velocity dims");
  static_assert(SD == 0 || USE_LDS, "split dims need the LDS variant");
  static_assert(LD == 0 || (LD == 1 && USE_LDS), "looped pencils need the LDS variant");
  constexpr int NF = D - RD - SD;     // fast (pencil-indexing) dims
  constexpr int ND = ipow(N, D);      // nodes per cell
  constexpr int T = ipow(N, NF);      // pencils per unit
  constexpr int CL = ipow(N, LD);     // pencils per thread
  constexpr int TT = T / CL;          // threads per unit
  constexpr int NS = ipow(N, RD);     // nodes per pencil
  constexpr int NU = ipow(N, SD);     // units (slabs) per cell
  constexpr int SST = ipow(N, NF + SD);  // node stride of the first register dim
  constexpr int UN = T * NS;          // nodes per unit
  static_assert(DX <= NF, "all x dims are fast dims");
  constexpr bool NT = (OPT & kOptStream) != 0;
  // FP32 mode keeps the FP64 input for the update when a thread owns few
  // nodes (else it is re-read: registers are scarce).
  constexpr bool KEEPU = sizeof(P) == 4 && NS <= 8 && LD == 0;

  unsigned cell, t0, lc = 0, unit = 0;
  if constexpr (USE_LDS) {
    lc = tid / TT;
    t0 = tid - lc * TT;
    const unsigned U = tile * prm.cells_per_wg + lc;
    cell = U / NU;
    unit = U - cell * NU;
  } else {
    const uint64_t p = (uint64_t)tile * blockDim.x + tid;
    cell = (unsigned)(p / T);
    t0 = (unsigned)(p - (uint64_t)cell * T);
  }
  // (Threads beyond cells_per_wg units of a workgroup, if any, stay
  // inactive.)
  const bool active = cell < prm.ncells && (!USE_LDS || lc < prm.cells_per_wg);
  if constexpr (!USE_LDS) {
    if (!active) return;
  }
  const unsigned cl = active ? cell : 0u;

  // Cell multi-index.
  unsigned c[D];
#pragma unroll
  for (int j = 0; j < D; ++j) c[j] = (cl / prm.cstride[j]) % prm.cells[j];
  // Fast node digits of pencil f.
  auto digits = [&](unsigned f, int *fd) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      fd[j] = (int)(f % N);
      f /= N;
    }
  };
  int fd0[NF > 0 ? NF : 1];
  if constexpr (LD == 0) digits(t0, fd0);

  // Split digits of this unit and the unit's node offset in the cell.
  int sd[SD > 0 ? SD : 1];
  unsigned soff = 0;
  {
    unsigned r = unit;
#pragma unroll
    for (int k = 0; k < SD; ++k) {
      sd[k] = (int)(r % N);
      r /= N;
      soff += (unsigned)sd[k] * (unsigned)ipow(N, NF + k);
    }
  }

  const uint64_t base0 = (uint64_t)cl * ND + t0 + soff;
  P u[NS];
  double u64[KEEPU ? NS : 1];
  if constexpr (LD == 0) {
    const uint64_t base = base0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double x = prm.u_in[base + (uint64_t)s * SST];
      if constexpr (KEEPU) u64[s] = x;
      u[s] = to_p<P>(x);
    }
  }
  const bool stage = prm.mode == 1;
  if constexpr (USE_LDS) {
    if constexpr (LD == 0) {
      if (lds_reuse) __syncthreads();
      if (active) {
#pragma unroll
        for (int s = 0; s < NS; ++s) lds[lc * UN + t0 + s * T] = u[s];
      }
    } else {
      // All pencils of this thread (the compiler issues loads ahead of the
      // stores as far as registers allow).
      const uint64_t base = (uint64_t)cl * ND + t0 + soff;
      if (lds_reuse) __syncthreads();
      if (active) {
#pragma unroll
        for (int q = 0; q < CL; ++q)
#pragma unroll
          for (int s = 0; s < NS; ++s)
            lds[lc * UN + t0 + q * TT + s * T] = to_p<P>(prm.u_in[base + q * TT + (uint64_t)s * SST]);
      }
    }
    __syncthreads();
    if (!active) return;
  }

  // The pencil f of this thread: field, sweeps, faces, update.
  auto pencil = [&](const unsigned f, const int *fd, const uint64_t base)
                    __attribute__((always_inline)) {
  if constexpr (LD == 1) {
#pragma unroll
    for (int s = 0; s < NS; ++s) u[s] = lds[lc * UN + f + s * T];
  }

  // Field at this thread's nodes. x dims are all fast, so E is per thread.
  P ev[DV];
  P vth[DX];   // velocity for x-dim j if its velocity dim is fast or split
  P vbase[DX]; // lo + c h for x-dim j if its velocity dim is a register dim
  const bool phase = prm.field_kind == 1;
  if (phase) {
    unsigned xcell = 0, xs = 1, xnode = 0, ns = 1;
#pragma unroll
    for (int m = 0; m < DX; ++m) {
      xcell += c[m] * xs;
      xs *= prm.cells[m];
      xnode += fd[m] * ns;
      ns *= N;
    }
    const P *e = prm.E + ((uint64_t)xcell * ipow(N, DX) + xnode) * DX;
#pragma unroll
    for (int j = 0; j < DV; ++j) ev[j] = prm.esign * e[j];
#pragma unroll
    for (int j = 0; j < DX; ++j) {
      const int m = DX + j;
      vbase[j] = prm.vlo[m] + P(c[m]) * prm.vh[m];
      if (m < NF) vth[j] = vbase[j] + prm.xi[fd[m]] * prm.vh[m];
      else if (m < NF + SD) vth[j] = vbase[j] + prm.xi[sd[m - NF]] * prm.vh[m];
      else vth[j] = P(0);
    }
  } else {
#pragma unroll
    for (int j = 0; j < DV; ++j) ev[j] = prm.a_const[DX + j];
#pragma unroll
    for (int j = 0; j < DX; ++j) {
      vth[j] = prm.a_const[j];
      vbase[j] = prm.a_const[j];
    }
  }
  // a_j at the thread's node s (compile-time j and s after unrolling).
  auto a_at = [&](int j, int s) -> P {
    if (j >= DX) return ev[j - DX];
    const int m = DX + j;
    if (!phase || m < NF + SD) return vth[j];
    const int r = m - NF - SD;
    const int dig = (s / ipow(N, r)) % N;
    return vbase[j] + prm.xi[dig] * prm.vh[m];
  };

  P acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = P(0);

  // Inflow-face loads are issued as unconditional batches (no branches
  // around them): a node off the inflow face reads its own value, a cache
  // hit, and gives it zero weight. Batching lets the loads of one
  // dimension overlap the volume sweep that follows them.
  // ---- slow (register) dimensions: face loads first ----
  constexpr int NL = NS / N;  // lines per register dimension
  P nbs[RD][NL];
#pragma unroll
  for (int r = 0; r < RD; ++r) {
    const int j = NF + SD + r;
    const int sstride = ipow(N, r);
    const unsigned cj = c[j], nj = prm.cells[j], st = prm.cstride[j];
    const unsigned left = cj == 0 ? cl + (nj - 1) * st : cl - st;
    const unsigned right = cj == nj - 1 ? cl - (nj - 1) * st : cl + st;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int s = (l % sstride) + (l / sstride) * sstride * N;  // digit r = 0
      const int sk = s + (N - 1) * sstride;
      const P a = a_at(j, s);
      const bool useL = a > P(0), useR = a < P(0);
      const unsigned cc = useL ? left : (useR ? right : cl);
      const int sn = useL ? sk : s;
      nbs[r][l] = to_p<P>(prm.u_in[(uint64_t)cc * ND + f + soff + (uint64_t)sn * SST]);
    }
  }
  constexpr bool kPrefetchDu = sizeof(P) == 4 || NS <= 4;
  P dv[NS];
  if (kPrefetchDu && stage && prm.read_du) {
#pragma unroll
    for (int s = 0; s < NS; ++s) dv[s] = ld_opt<NT>(prm.du + base + (uint64_t)s * SST);
  }
  sched_fence();

  // ---- fast (thread-distributed) dimensions ----
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    const int ij = fd[j];
    const int stride = ipow(N, j);
    const unsigned cj = c[j], nj = prm.cells[j], st = prm.cstride[j];
    const unsigned left = cj == 0 ? cl + (nj - 1) * st : cl - st;
    const unsigned right = cj == nj - 1 ? cl - (nj - 1) * st : cl + st;
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = prm.Dm[ij * N + m];
    const int off0 = (int)f - ij * stride;  // node offset of digit j = 0
    const P ih = prm.inv_h[j];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      P sum = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) {
        P v;
        if constexpr (USE_LDS) v = lds[lc * UN + off0 + m * stride + s * T];
        else v = to_p<P>(prm.u_in[(uint64_t)cl * ND + off0 + m * stride + (uint64_t)s * T]);
        sum += row[m] * v;
      }
      acc[s] -= a_at(j, s) * ih * sum;
    }
    // Inflow face: the only place the neighbour's trace enters. Only
    // threads on a face of this dimension take part; their loads are
    // issued as one batch before any is used.
    if (ij == 0 || ij == N - 1) {
      const bool onL = ij == 0, onR = ij == N - 1;
      P nb[NS];
  #pragma unroll
      for (int s = 0; s < NS; ++s) {
        const P a = a_at(j, s);
        const bool useL = onL && a > P(0), useR = onR && a < P(0);
        const unsigned cc = useL ? left : (useR ? right : cl);
        const int node = (int)f + (useL ? (N - 1) * stride : (useR ? -(N - 1) * stride : 0));
        nb[s] = to_p<P>(prm.u_in[(uint64_t)cc * ND + soff + node + (uint64_t)s * SST]);
      }
      const P lf = prm.lift_inv_h[j];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const P a = a_at(j, s);
        const bool useL = onL && a > P(0), useR = onR && a < P(0);
        const P w = useL ? lf * a : (useR ? -lf * a : P(0));
        acc[s] += w * (nb[s] - u[s]);
      }
    }
    sched_fence();
  }

  // ---- split dimensions: the other slabs of the line from global memory ----
#pragma unroll
  for (int k = 0; k < SD; ++k) {
    const int j = NF + k;
    const int stride = ipow(N, j);
    const int ij = sd[k];
    const unsigned cj = c[j], nj = prm.cells[j], st = prm.cstride[j];
    const unsigned left = cj == 0 ? cl + (nj - 1) * st : cl - st;
    const unsigned right = cj == nj - 1 ? cl - (nj - 1) * st : cl + st;
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = prm.Dm[ij * N + m];
    const uint64_t line0 = (uint64_t)cl * ND + f + soff - (unsigned)(ij * stride);
    const P ih = prm.inv_h[j];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      P v[N];
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = to_p<P>(prm.u_in[line0 + m * stride + (uint64_t)s * SST]);
      P sum = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) sum += row[m] * v[m];
      acc[s] -= a_at(j, s) * ih * sum;
    }
    if (ij == 0 || ij == N - 1) {
      const bool onL = ij == 0, onR = ij == N - 1;
      P nb[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const P a = a_at(j, s);
        const bool useL = onL && a > P(0), useR = onR && a < P(0);
        const unsigned cc = useL ? left : (useR ? right : cl);
        const int node = (int)(f + soff) + (useL ? (N - 1) * stride : (useR ? -(N - 1) * stride : 0));
        nb[s] = to_p<P>(prm.u_in[(uint64_t)cc * ND + node + (uint64_t)s * SST]);
      }
      const P lf = prm.lift_inv_h[j];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const P a = a_at(j, s);
        const bool useL = onL && a > P(0), useR = onR && a < P(0);
        const P w = useL ? lf * a : (useR ? -lf * a : P(0));
        acc[s] += w * (nb[s] - u[s]);
      }
    }
    sched_fence();
  }

  // ---- slow (register) dimensions ----
#pragma unroll
  for (int r = 0; r < RD; ++r) {
    const int j = NF + SD + r;
    const int sstride = ipow(N, r);
    const P ih = prm.inv_h[j];
    const P lf = prm.lift_inv_h[j];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int ij = (s / sstride) % N;
      const int s0 = s - ij * sstride;
      P sum = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) sum += prm.Dm[ij * N + m] * u[s0 + m * sstride];
      acc[s] -= a_at(j, s) * ih * sum;
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int s = (l % sstride) + (l / sstride) * sstride * N;
      const int sk = s + (N - 1) * sstride;
      const P a = a_at(j, s);
      const P wL = a > P(0) ? lf * a : P(0);
      const P wR = a < P(0) ? -lf * a : P(0);
      acc[s] += wL * (nbs[r][l] - u[s]);
      acc[sk] += wR * (nbs[r][l] - u[sk]);
    }
  }

  // ---- output ----
  if (!stage) {
#pragma unroll
    for (int s = 0; s < NS; ++s) prm.out[base + (uint64_t)s * SST] = acc[s];
    return;
  }
  // FP64 with many nodes per thread reads the increment only now, keeping
  // registers free during the sweeps.
  if (prm.read_du) {
    if (!kPrefetchDu) {
#pragma unroll
      for (int s = 0; s < NS; ++s) dv[s] = ld_opt<NT>(prm.du + base + (uint64_t)s * SST);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) dv[s] = rk_fma(prm.rk_a, dv[s], prm.dt * acc[s]);
  } else {
#pragma unroll
    for (int s = 0; s < NS; ++s) dv[s] = prm.dt * acc[s];
  }
  if (prm.write_du) {
#pragma unroll
    for (int s = 0; s < NS; ++s) st_opt<NT>(prm.du + base + (uint64_t)s * SST, dv[s]);
  }
  // FP64 solution update (FP32 mode: the kept or re-read FP64 input).
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double uo;
    if constexpr (sizeof(P) == sizeof(double)) uo = (double)u[s];
    else if constexpr (KEEPU) uo = u64[s];
    else uo = prm.u_in[base + (uint64_t)s * SST];
    st_opt<NT>(prm.u_out + base + (uint64_t)s * SST, rk_fma(prm.rk_b, (double)dv[s], uo));
  }
  };  // pencil
  if constexpr (LD == 0) {
    pencil(t0, fd0, base0);
  } else {
#pragma unroll 1
    for (int q = 0; q < CL; ++q) {
      int fd[NF > 0 ? NF : 1];
      digits(t0 + q * TT, fd);
      pencil(t0 + q * TT, fd, base0 + q * TT);
    }
  }
}

template <int D, int N, int DX, int RD, typename P, bool USE_LDS, int SD, int OPT, int LD = 0>
__global__ void __launch_bounds__((stage_max_threads<D, N, RD, USE_LDS, SD, LD>()))
    stage_kernel(const StageParams<P> prm) {
  extern __shared__ unsigned char smem_raw[];
  unsigned tile = blockIdx.x;
  if (prm.xcd_remap) tile = xcd_tile(tile, prm.nblocks);
  stage_body<D, N, DX, RD, P, USE_LDS, SD, OPT, LD>(prm, tile, reinterpret_cast<P *>(smem_raw),
                                                    false, threadIdx.x);
}

// Work list of a batched launch (work_list.h): the solves of one launch
// group (one compiled variant and launch shape) in slots 0..nslots-1, a
// solve's tile count in its StageParams::nblocks.
// A solve's parameters as the work-list kernels read them: in the constant
// address space, so the loads are scalar and invariant, like those of a
// kernel argument.
template <typename P>
using ConstStageParams = const __attribute__((address_space(4))) StageParams<P>;

template <typename P>
struct ListParams {
  ConstStageParams<P> *prm;  // one per slot
  const uint32_t *item0;     // nslots + 1 entries (work_list.h)
  int nslots;
  unsigned nitems;           // item0[nslots] = the grid
};

// Work-list form of stage_kernel: one launch covers the tiles of every solve
// of a group, workgroup `item` running the stage body of the item's solve
// and tile with that solve's parameters. (A form in which each workgroup
// loops over items holds the body's registers across iterations: the
// compiler gives it fewer waves per SIMD than stage_kernel for a quarter of
// the variants, so the work items are workgroups here.)
template <int D, int N, int DX, int RD, typename P, bool USE_LDS, int SD, int OPT, int LD = 0>
__global__ void __launch_bounds__((stage_max_threads<D, N, RD, USE_LDS, SD, LD>()))
    stage_list_kernel(const ListParams<P> lp) {
  extern __shared__ unsigned char smem_raw[];
  const unsigned item = blockIdx.x;
  const int slot = __builtin_amdgcn_readfirstlane(work_list_slot(lp.item0, lp.nslots, item));
  const unsigned t0 = __builtin_amdgcn_readfirstlane(item - lp.item0[slot]);
  ConstStageParams<P> &prm = lp.prm[slot];
  if (t0 >= prm.nblocks) return;  // padding: the whole workgroup
  const unsigned tile = prm.xcd_remap ? xcd_tile(t0, prm.nblocks) : t0;
  stage_body<D, N, DX, RD, P, USE_LDS, SD, OPT, LD, ConstStageParams<P>>(
      prm, tile, reinterpret_cast<P *>(smem_raw), false, threadIdx.x);
}

}  // namespace hd
