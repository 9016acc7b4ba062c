// Fused LSRK stage with Gauss-Legendre quadrature (Sec. 2.5, the paper's
// default rule: k+1 Gauss points per dimension, GL nodal basis).
//
// With B[q][i] = l_i(g_q) square and invertible, the exactly integrated mass
// matrix is M = B^T diag(W |J|) B in tensor form, so M^{-1} = B^{-1}
// diag^{-1} B^{-T} also factorizes over dimensions, and the stage operator
// can be evaluated entirely at the Gauss points (Cartesian cells, fields with
// a_j independent of x_j, strong form which equals the weak form here since
// the rule integrates the by-parts identity along each line exactly):
//   U = (B x ... x B) u                                     (d sweeps)
//   Y(q) = - sum_j a_j(q) / h_j (Dg_j U)(q)                 (Dg = B' B^{-1})
//        + sum_faces lift_s[q_j] / h_j min(a.n, 0)(p) (u_own - u_nbr)(p)
//   L(u) = (B^{-1} x ... x B^{-1}) Y                        (d sweeps)
// where p is q's tangential part, u_own(p) = sum_m ext_s[m] U(.., m, ..) is
// the own trace at the face's Gauss points, u_nbr the neighbour's nodal face
// layer carried to them by d-1 tangential sweeps, and lift_s = B^{-T} e_s /
// omega. With GL points (B = I) this is the collocation operator.
//
// One workgroup per cell; everything is a sweep over lines in LDS: the
// cell's values at the Gauss points, the operator accumulated beside them,
// one face layer at a time.
#pragma once

#include <hip/hip_runtime.h>

#include "stage_kernel.h"

namespace hd {

template <typename P>
struct GaussTables {
  P B[kMaxN * kMaxN];
  P Binv[kMaxN * kMaxN];
  P Dg[kMaxN * kMaxN];
  P ext[2][kMaxN];
  P lift[2][kMaxN];
  P g[kMaxN];
  P om[kMaxN];
};

// Up to 1024 threads: few nodes per thread keep the per-node registers (the
// accumulated stage operator, u and du) small.
constexpr int gauss_threads(int nd) { return nd >= 256 ? 256 : (nd + 63) / 64 * 64; }

// Elements of the 1D tables (B, B^{-1}, Dg, ext, lift, g, om).
constexpr int gauss_table_elems(int n) { return 3 * n * n + 6 * n; }

// Metric of a mapped x-cell (the tensor-product mapping keeps it in x-space:
// O(#x-cells) storage, combined with the Cartesian v-metric on the fly):
// at each x-quadrature point xq, adj(A) (dx x dx, row-major) and det(A) for
// A = d x / d xi of the x-block; then, for each x-dimension j and side s, at
// the face's tangential x-points, row j of adj(A) on that face.
constexpr int gauss_metric_elems(int n, int dx) {
  return ipow(n, dx) * (dx * dx + 1) + dx * 2 * ipow(n, dx - 1) * dx;
}

// LDS arrays are padded by one element after every n^2: a thread's n x n
// plane then starts n^2 + 1 elements after its neighbour's, which spreads
// the lanes of a sweep over the banks.
template <int N>
__host__ __device__ constexpr int gauss_pad(int q) { return q + q / (N * N); }
constexpr int gauss_padded(int n, int count) { return count + count / (n * n) + 1; }

// Where mapped cells read their metric: FP32 stages it in LDS; FP64 reads it
// from global memory (a few KiB per x-cell, shared by every velocity cell,
// so cache hits), because in LDS it would cost the FP64 6D degree-3 kernel
// its second workgroup per CU (measured: 103 against 58 ms per stage),
// while FP32 is held to 3 waves per SIMD by registers and loses 10% on the
// global reads.
constexpr bool gauss_metric_in_lds(int psize) { return psize == 4; }

// LDS elements of P: U and the accumulator Y (n^d each), one face layer,
// E at the x-Gauss points, the 1D tables and, for mapped cells in FP32, the
// metric.
constexpr int gauss_lds_elems(int d, int n, int dx, bool mapped, int psize) {
  return 2 * gauss_padded(n, ipow(n, d)) + gauss_padded(n, ipow(n, d - 1)) + ipow(n, dx) * dx +
         gauss_table_elems(n) +
         (mapped && gauss_metric_in_lds(psize) ? gauss_metric_elems(n, dx) : 0);
}

// Even-odd form (Sec. 2.6, sum factorization) of an N x N matrix M that is
// centro-symmetric, M[N-1-q][N-1-m] = M[q][m] (the interpolation between
// the symmetric Gauss-Lobatto nodes and Gauss points, and its inverse), or
// with ANTI centro-antisymmetric, M[N-1-q][N-1-m] = -M[q][m] (the derivative
// at the Gauss points). With the sums e_m = v_m + v_{N-1-m} and differences
// o_m = v_m - v_{N-1-m} (m < h = N/2; e also holds the middle value v_h for
// odd N), row q < h of M v splits into E_q = sum_m ME[q][m] e_m and
// O_q = sum_m MO[q][m] o_m, ME and MO the half sums and half differences of
// M[q][m] and M[q][N-1-m]:
//   (M v)_q = E_q + O_q,  (M v)_{N-1-q} = E_q - O_q  (ANTI: O_q - E_q),
// and the middle row of odd N is sum_m M[h][m] e_m (ANTI: sum_m M[h][m] o_m;
// its diagonal entry vanishes). About N^2 / 2 + 2 N operations per line
// instead of N^2: 30 against 36 at N = 6, 21 against 25 at N = 5; none saved
// below N = 5, where the dense form stays.
template <int N, typename P>
struct GaussEvenOdd {
  static constexpr int H = N / 2, HE = (N + 1) / 2;
  P me[H > 0 ? H : 1][HE];
  P mo[H > 0 ? H : 1][H > 0 ? H : 1];
  P mid[HE];  // middle row of odd N
};

template <int N, bool ANTI, typename P>
__device__ __forceinline__ void gauss_eo_make(const P *M, GaussEvenOdd<N, P> &c) {
  constexpr int H = N / 2, HE = (N + 1) / 2;
#pragma unroll
  for (int q = 0; q < H; ++q) {
#pragma unroll
    for (int m = 0; m < H; ++m) {
      c.me[q][m] = P(0.5) * (M[q * N + m] + M[q * N + N - 1 - m]);
      c.mo[q][m] = P(0.5) * (M[q * N + m] - M[q * N + N - 1 - m]);
    }
    if constexpr (HE > H) c.me[q][H] = M[q * N + H];
  }
  if constexpr (HE > H) {
#pragma unroll
    for (int m = 0; m < HE; ++m) c.mid[m] = M[H * N + m];
  }
}

template <int N, bool ANTI, typename P>
__device__ __forceinline__ void gauss_eo_apply(const GaussEvenOdd<N, P> &c, P (&v)[N]) {
  constexpr int H = N / 2, HE = (N + 1) / 2;
  P e[HE], o[H > 0 ? H : 1];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = v[m] + v[N - 1 - m];
    o[m] = v[m] - v[N - 1 - m];
  }
  if constexpr (HE > H) e[H] = v[H];
#pragma unroll
  for (int q = 0; q < H; ++q) {
    P E = c.me[q][0] * e[0], O = c.mo[q][0] * o[0];
#pragma unroll
    for (int m = 1; m < HE; ++m) E += c.me[q][m] * e[m];
#pragma unroll
    for (int m = 1; m < H; ++m) O += c.mo[q][m] * o[m];
    v[q] = E + O;
    v[N - 1 - q] = ANTI ? O - E : E - O;
  }
  if constexpr (HE > H) {
    if constexpr (ANTI) {
      P E = c.mid[0] * o[0];
#pragma unroll
      for (int m = 1; m < H; ++m) E += c.mid[m] * o[m];
      v[H] = E;
    } else {
      P E = c.mid[0] * e[0];
#pragma unroll
      for (int m = 1; m < HE; ++m) E += c.mid[m] * e[m];
      v[H] = E;
    }
  }
}

// The transforms of lines use the even-odd form from N = 5 on.
template <int N>
constexpr bool gauss_use_eo() { return N >= 5; }

// In place along one axis (stride = N^axis) of an N-ary array of `total`
// elements: every line v <- M v (M one of the interpolation matrices).
template <int N, typename P>
__device__ __forceinline__ void gauss_sweep(P *buf, int total, int stride, const P *M, int t,
                                            int T) {
  const int lines = total / N;
  GaussEvenOdd<N, P> c;
  if constexpr (gauss_use_eo<N>()) gauss_eo_make<N, false>(M, c);
  for (int l = t; l < lines; l += T) {
    const int lo = l % stride, hi = l / stride;
    const int base = lo + hi * stride * N;
    P v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = buf[gauss_pad<N>(base + m * stride)];
    if constexpr (gauss_use_eo<N>()) {
      gauss_eo_apply<N, false>(c, v);
#pragma unroll
      for (int q = 0; q < N; ++q) buf[gauss_pad<N>(base + q * stride)] = v[q];
    } else {
#pragma unroll
      for (int q = 0; q < N; ++q) {
        P s = M[q * N] * v[0];
#pragma unroll
        for (int m = 1; m < N; ++m) s += M[q * N + m] * v[m];
        buf[gauss_pad<N>(base + q * stride)] = s;
      }
    }
  }
}

// In place along two adjacent axes (strides st and st * N) of an N-ary
// array: every N x N plane v <- M v M^T, kept in registers between the two
// passes (one barrier for two dimensions).
template <int N, typename P>
__device__ __forceinline__ void gauss_sweep2(P *buf, int total, int st, const P *M, int t,
                                             int T) {
  const int planes = total / (N * N);
  GaussEvenOdd<N, P> c;
  if constexpr (gauss_use_eo<N>()) gauss_eo_make<N, false>(M, c);
  for (int l = t; l < planes; l += T) {
    const int lo = l % st, hi = l / st;
    const int base = lo + hi * st * N * N;
    P v[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = 0; b < N; ++b) v[a][b] = buf[gauss_pad<N>(base + a * st + b * st * N)];
    if constexpr (gauss_use_eo<N>()) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        P w[N];
#pragma unroll
        for (int q = 0; q < N; ++q) w[q] = v[q][b];
        gauss_eo_apply<N, false>(c, w);
#pragma unroll
        for (int q = 0; q < N; ++q) v[q][b] = w[q];
      }
#pragma unroll
      for (int a = 0; a < N; ++a) {
        gauss_eo_apply<N, false>(c, v[a]);
#pragma unroll
        for (int q = 0; q < N; ++q) buf[gauss_pad<N>(base + a * st + q * st * N)] = v[a][q];
      }
      continue;
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
      P w[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        P s = M[q * N] * v[0][b];
#pragma unroll
        for (int m = 1; m < N; ++m) s += M[q * N + m] * v[m][b];
        w[q] = s;
      }
#pragma unroll
      for (int q = 0; q < N; ++q) v[q][b] = w[q];
    }
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        P s = M[q * N] * v[a][0];
#pragma unroll
        for (int m = 1; m < N; ++m) s += M[q * N + m] * v[a][m];
        buf[gauss_pad<N>(base + a * st + q * st * N)] = s;
      }
  }
}

// All DIMS axes of an N^DIMS array, two at a time.
template <int N, int DIMS, typename P>
__device__ __forceinline__ void gauss_transform(P *buf, const P *M, int t, int T) {
  constexpr int total = ipow(N, DIMS);
#pragma unroll
  for (int a = 0; a + 1 < DIMS; a += 2) {
    gauss_sweep2<N>(buf, total, ipow(N, a), M, t, T);
    __syncthreads();
  }
  if constexpr (DIMS % 2 == 1) {
    gauss_sweep<N>(buf, total, ipow(N, DIMS - 1), M, t, T);
    __syncthreads();
  }
}

// MAPPED: the weak form on mapped cells, with the contravariant flux
// ahat = |J| J^{-1} a at the quadrature points (the x-metric from the table,
// the v-metric diag(h)), upwind traces u* on every face, and the mass matrix
// with |J|:
//   Y(q) = [ sum_j sum_m Dg[m][q_j] om_m ahat_j U (along j) / om_{q_j}
//            - sum_s lift_s[q_j] (ahat_j n_s u*)(p) ] / |J(q)|,
// then L(u) = (B^{-1})^{x d} Y. The tables may be the collocation ones.
template <int D, int N, int DX, typename P, bool MAPPED = false>
__global__ void __launch_bounds__(gauss_threads(ipow(N, D)))
    stage_gauss_kernel(const StageParams<P> prm, const GaussTables<P> gt) {
  constexpr int ND = ipow(N, D), NF = ND / N, T = gauss_threads(ND);
  constexpr int NXN = ipow(N, DX);
  extern __shared__ __align__(16) unsigned char smem_raw[];  // 16: FP64 arrays after static LDS
  P *W = reinterpret_cast<P *>(smem_raw);      // the cell, then U
  P *Yb = W + gauss_padded(N, ND);             // the operator at the Gauss points, then L(u)
  P *F = Yb + gauss_padded(N, ND);             // one face layer
  P *EG = F + gauss_padded(N, NF);             // E at the x-Gauss points [xq][comp]
  // 1D tables in LDS, to be indexed per lane. One thread copies them with
  // compile-time indices: a kernel argument indexed per lane would be copied
  // whole to scratch.
  P *tB = EG + NXN * DX, *tBinv = tB + N * N, *tDg = tBinv + N * N;
  P *tExt = tDg + N * N, *tLift = tExt + 2 * N, *tG = tLift + 2 * N, *tOm = tG + N;
  constexpr int MXE = DX * DX + 1, NFX = NXN / N;
  const int t = threadIdx.x;
  if (t == 0) {
#pragma unroll
    for (int i = 0; i < N * N; ++i) {
      tB[i] = gt.B[i];
      tBinv[i] = gt.Binv[i];
      tDg[i] = gt.Dg[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      tExt[i] = gt.ext[0][i];
      tExt[N + i] = gt.ext[1][i];
      tLift[i] = gt.lift[0][i];
      tLift[N + i] = gt.lift[1][i];
      tG[i] = gt.g[i];
      tOm[i] = gt.om[i];
    }
  }
  unsigned cell = blockIdx.x;
  if (prm.xcd_remap) cell = xcd_tile(cell, prm.nblocks);

  unsigned c[D], left[D], right[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c[j] = (cell / prm.cstride[j]) % prm.cells[j];
    const unsigned nj = prm.cells[j], st = prm.cstride[j];
    left[j] = c[j] == 0 ? cell + (nj - 1) * st : cell - st;
    right[j] = c[j] == nj - 1 ? cell - (nj - 1) * st : cell + st;
  }
  const bool phase = prm.field_kind == 1;
  const bool stage = prm.mode == 1;
  const double *ucell = prm.u_in + (uint64_t)cell * ND;
  for (int q = t; q < ND; q += T) W[gauss_pad<N>(q)] = (P)ucell[q];
  unsigned xcell = 0, xs = 1;
#pragma unroll
  for (int m = 0; m < DX; ++m) {
    xcell += c[m] * xs;
    xs *= prm.cells[m];
  }
  P detv = P(1);
  // mapped cells: this x-cell's metric, [xq][MXE] then [j][side][face
  // x-point][DX], read from LDS (FP32) or global memory (FP64)
  constexpr bool ML = gauss_metric_in_lds(sizeof(P));
  const double *MXg = MAPPED ? prm.xmetric + (uint64_t)xcell * gauss_metric_elems(N, DX) : nullptr;
  P *MXl = tOm + N;
  auto metric = [&](int i) -> P {
    if constexpr (ML) return MXl[i];
    else return (P)MXg[i];
  };
  if constexpr (MAPPED) {
    if constexpr (ML)
      for (int i = t; i < gauss_metric_elems(N, DX); i += T) MXl[i] = (P)MXg[i];
#pragma unroll
    for (int m = DX; m < D; ++m) detv *= prm.vh[m];
  }
  __syncthreads();  // tables ready
  if (phase) {
    // E at the x-Gauss points: the nodal interpolant of the cell's E table
    const P *e = prm.E + (uint64_t)xcell * NXN * DX;
    for (int idx = t; idx < NXN * DX; idx += T) {
      const int xq = idx / DX, comp = idx % DX;
      P s = P(0);
      for (int xn = 0; xn < NXN; ++xn) {
        P ph = P(1);
        int a = xq, b = xn;
#pragma unroll
        for (int m = 0; m < DX; ++m) {
          ph *= tB[(a % N) * N + (b % N)];
          a /= N;
          b /= N;
        }
        s += ph * e[xn * DX + comp];
      }
      EG[idx] = prm.esign * s;
    }
  }
  // a_j at the point with index q (its digit j is not used: a_j does not
  // depend on x_j)
  auto a_at = [&](int j, int q) -> P {
    if (!phase) return prm.a_const[j];
    if (j < DX) {
      const int dv = (q / ipow(N, DX + j)) % N;
      return prm.vlo[DX + j] + (P(c[DX + j]) + tG[dv]) * prm.vh[DX + j];
    }
    return EG[(q % NXN) * DX + (j - DX)];
  };
  // ahat_j at the cell point q (mapped cells)
  auto ahat_at = [&](int j, int q) -> P {
    const int mx = (q % NXN) * MXE;
    if (j < DX) {
      P s = P(0);
#pragma unroll
      for (int k2 = 0; k2 < DX; ++k2) s += metric(mx + j * DX + k2) * a_at(k2, q);
      return detv * s;
    }
    return metric(mx + DX * DX) * detv * prm.inv_h[j] * a_at(j, q);
  };
  // ahat_j at the point with index q (digit j ignored) on face `side` of
  // dimension j
  auto ahat_face = [&](int j, int side, int q) -> P {
    if (j < DX) {
      const int sj = ipow(N, j), xq = q % NXN;
      const int xp = xq % sj + (xq / (sj * N)) * sj;
      const int mf = NXN * MXE + ((j * 2 + side) * NFX + xp) * DX;
      P s = P(0);
#pragma unroll
      for (int k2 = 0; k2 < DX; ++k2) s += metric(mf + k2) * a_at(k2, q);
      return detv * s;
    }
    return ahat_at(j, q);
  };
  // Which face sides have inflow Gauss points (bit 2 j + side), and the
  // neighbour layers of one such side per dimension loaded into registers
  // now, so that their latency overlaps the transform.
  // (Only while that holds at most 32 values per thread: beyond it the layers
  // would spill.)
  constexpr int RF = (NF + T - 1) / T;
  constexpr bool kPre = D * RF <= 32;
  __shared__ int active_mask;
  int active = 0;
  int pre_side[D];
  double pre[kPre ? D : 1][kPre ? RF : 1];
  {
    if (t == 0) active_mask = 0;
    __syncthreads();  // EG ready, mask cleared
    int mine = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = ipow(N, j);
      for (int p = t; p < NF; p += T) {
        const int q = p % sj + (p / sj) * sj * N;
        if constexpr (MAPPED && !kPre) {
          mine = (1 << (2 * D)) - 1;  // every side may have inflow points
        } else if constexpr (MAPPED) {
          mine |= (ahat_face(j, 0, q) > P(0) ? 1 : 0) << (2 * j);
          mine |= (ahat_face(j, 1, q) < P(0) ? 1 : 0) << (2 * j + 1);
        } else {
          const P a = a_at(j, q);
          mine |= (a > P(0) ? 1 : 0) << (2 * j);
          mine |= (a < P(0) ? 1 : 0) << (2 * j + 1);
        }
      }
    }
    if (mine) atomicOr(&active_mask, mine);
    __syncthreads();
    active = active_mask;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = ipow(N, j);
      pre_side[j] = (active >> (2 * j)) & 1 ? 0 : ((active >> (2 * j + 1)) & 1 ? 1 : -1);
      if constexpr (!kPre) pre_side[j] = -1;
      if (pre_side[j] < 0) continue;
      const double *un = prm.u_in + (uint64_t)(pre_side[j] ? right[j] : left[j]) * ND;
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int p = t + T * r;
        const int node = p % sj + (pre_side[j] ? 0 : N - 1) * sj + (p / sj) * sj * N;
        pre[kPre ? j : 0][kPre ? r : 0] = p < NF ? un[node] : 0.0;
      }
    }
  }
  // U = (B x ... x B) u
  gauss_transform<N, D>(W, tB, t, T);


  if constexpr (MAPPED) {
    // volume (weak form), one dimension per sweep; Dg^T is centro-
    // antisymmetric like Dg
    GaussEvenOdd<N, P> dte;
    if constexpr (gauss_use_eo<N>()) {
      P mt[N * N];
#pragma unroll
      for (int q = 0; q < N; ++q)
#pragma unroll
        for (int m = 0; m < N; ++m) mt[q * N + m] = tDg[m * N + q];
      gauss_eo_make<N, true>(mt, dte);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = ipow(N, j);
      for (int l = t; l < NF; l += T) {
        const int base = l % sj + (l / sj) * sj * N;
        P tv[N];
#pragma unroll
        for (int m = 0; m < N; ++m)
          tv[m] = tOm[m] * ahat_at(j, base + m * sj) * W[gauss_pad<N>(base + m * sj)];
        if constexpr (gauss_use_eo<N>()) gauss_eo_apply<N, true>(dte, tv);
#pragma unroll
        for (int qq = 0; qq < N; ++qq) {
          P s;
          if constexpr (gauss_use_eo<N>()) {
            s = tv[qq];
          } else {
            s = tDg[qq] * tv[0];
#pragma unroll
            for (int m = 1; m < N; ++m) s += tDg[m * N + qq] * tv[m];
          }
          s /= tOm[qq];
          if (j == 0) Yb[gauss_pad<N>(base + qq * sj)] = s;
          else Yb[gauss_pad<N>(base + qq * sj)] += s;
        }
      }
      __syncthreads();
    }
    // faces: every side contributes - lift (ahat.n) u*
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = ipow(N, j);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const bool nbr = (active >> (2 * j + side)) & 1;
        if (nbr) {
          if (side == pre_side[j]) {
#pragma unroll
            for (int r = 0; r < RF; ++r) {
              const int p = t + T * r;
              if (p < NF) F[gauss_pad<N>(p)] = (P)pre[kPre ? j : 0][kPre ? r : 0];
            }
          } else {
            const double *un = prm.u_in + (uint64_t)(side ? right[j] : left[j]) * ND;
            for (int p = t; p < NF; p += T) {
              const int node = p % sj + (side ? 0 : N - 1) * sj + (p / sj) * sj * N;
              F[gauss_pad<N>(p)] = (P)un[node];
            }
          }
          __syncthreads();
          gauss_transform<N, D - 1>(F, tB, t, T);
        }
        for (int p = t; p < NF; p += T) {
          const int base = p % sj + (p / sj) * sj * N;
          P uo = P(0);
#pragma unroll
          for (int m = 0; m < N; ++m) uo += tExt[side * N + m] * W[gauss_pad<N>(base + m * sj)];
          const P a = ahat_face(j, side, base);
          const P an = side ? a : -a;
          const P us = (an >= P(0) || !nbr) ? uo : F[gauss_pad<N>(p)];
          F[gauss_pad<N>(p)] = an * us;
        }
        __syncthreads();
        for (int q = t; q < ND; q += T) {
          const int qj = (q / sj) % N;
          const int p = q % sj + (q / (sj * N)) * sj;
          Yb[gauss_pad<N>(q)] -= tLift[side * N + qj] * F[gauss_pad<N>(p)];
        }
        __syncthreads();
      }
    }
    // inverse of |J|
    for (int q = t; q < ND; q += T) Yb[gauss_pad<N>(q)] /= metric((q % NXN) * MXE + DX * DX) * detv;
    __syncthreads();
  } else {
    // Per dimension j: the faces' scaled upwind jumps at their Gauss points,
    // then one sweep along j that adds the volume term - a_j / h_j Dg_j U
    // and lifts the jump into Y (a lift spreads along j only). When both
    // sides have inflow points, the first is lifted in a pass of its own.
    bool ystarted = false;  // Y has been written (uniform)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = ipow(N, j);
      const P ih = prm.inv_h[j];
      int pending = -1;  // side whose jumps wait in F for the sweep (uniform)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        // A side none of whose Gauss points is inflow contributes nothing.
        if (!((active >> (2 * j + side)) & 1)) continue;
        if (pending >= 0) {
          for (int q = t; q < ND; q += T) {
            const int qj = (q / sj) % N;
            const int p = q % sj + (q / (sj * N)) * sj;
            const P y = ih * tLift[pending * N + qj] * F[gauss_pad<N>(p)];
            if (ystarted) Yb[gauss_pad<N>(q)] += y;
            else Yb[gauss_pad<N>(q)] = y;
          }
          ystarted = true;
          __syncthreads();
        }
        // side 0 (face xi_j = 0): the left neighbour's layer i_j = k;
        // side 1 (xi_j = 1): the right neighbour's layer i_j = 0. The layer
        // of the prefetched side is already in registers.
        if (side == pre_side[j]) {
#pragma unroll
          for (int r = 0; r < RF; ++r) {
            const int p = t + T * r;
            if (p < NF) F[gauss_pad<N>(p)] = (P)pre[kPre ? j : 0][kPre ? r : 0];
          }
        } else {
          const double *un = prm.u_in + (uint64_t)(side ? right[j] : left[j]) * ND;
          for (int p = t; p < NF; p += T) {
            const int node = p % sj + (side ? 0 : N - 1) * sj + (p / sj) * sj * N;
            F[gauss_pad<N>(p)] = (P)un[node];
          }
        }
        __syncthreads();
        gauss_transform<N, D - 1>(F, tB, t, T);
        for (int p = t; p < NF; p += T) {
          const int base = p % sj + (p / sj) * sj * N;
          P uo = P(0);
#pragma unroll
          for (int m = 0; m < N; ++m) uo += tExt[side * N + m] * W[gauss_pad<N>(base + m * sj)];
          const P a = a_at(j, base);
          const P an = side ? a : -a;
          F[gauss_pad<N>(p)] = (an < P(0) ? an : P(0)) * (uo - F[gauss_pad<N>(p)]);
        }
        __syncthreads();
        pending = side;
      }
      // the sweep along j: line l has the tangential index l of the layer
      GaussEvenOdd<N, P> dge;
      if constexpr (gauss_use_eo<N>()) gauss_eo_make<N, true>(tDg, dge);
      for (int l = t; l < NF; l += T) {
        const int base = l % sj + (l / sj) * sj * N;
        P v[N];
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = W[gauss_pad<N>(base + m * sj)];
        const P coef = -a_at(j, base) * ih;
        const P fj = pending >= 0 ? ih * F[gauss_pad<N>(l)] : P(0);
        if constexpr (gauss_use_eo<N>()) gauss_eo_apply<N, true>(dge, v);
#pragma unroll
        for (int qq = 0; qq < N; ++qq) {
          P s;
          if constexpr (gauss_use_eo<N>()) {
            s = v[qq];
          } else {
            s = tDg[qq * N] * v[0];
#pragma unroll
            for (int m = 1; m < N; ++m) s += tDg[qq * N + m] * v[m];
          }
          P y = coef * s;
          if (pending >= 0) y += tLift[pending * N + qq] * fj;
          const int q = gauss_pad<N>(base + qq * sj);
          if (ystarted) Yb[q] += y;
          else Yb[q] = y;
        }
      }
      ystarted = true;
      __syncthreads();  // Y complete for this dimension; F is free again
    }
  }  // Cartesian cells
  // L(u) = (B^{-1} x ... x B^{-1}) Y
  gauss_transform<N, D>(Yb, tBinv, t, T);

  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
    for (int q = t; q < ND; q += T) ocell[q] = Yb[gauss_pad<N>(q)];
    return;
  }
  P *ducell = prm.du + (uint64_t)cell * ND;
  double *uocell = prm.u_out + (uint64_t)cell * ND;
  for (int q = t; q < ND; q += T) {
    const P L = Yb[gauss_pad<N>(q)];
    const P dn = prm.read_du ? prm.rk_a * ducell[q] + prm.dt * L : prm.dt * L;
    if (prm.write_du) ducell[q] = dn;
    uocell[q] = ucell[q] + prm.rk_b * (double)dn;
  }
}

}  // namespace hd
