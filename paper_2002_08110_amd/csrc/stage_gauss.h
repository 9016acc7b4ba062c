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
// One workgroup per cell; the cell is transformed in place in LDS.
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
};

constexpr int gauss_threads(int nd) { return nd >= 256 ? 256 : (nd + 63) / 64 * 64; }

// LDS elements of P: the cell, two face layers, E at the x-Gauss points.
constexpr int gauss_lds_elems(int d, int n, int dx) {
  return ipow(n, d) + 2 * ipow(n, d - 1) + ipow(n, dx) * dx;
}

// In place along one axis (stride = N^axis) of consecutive N-ary arrays of
// `total` elements: every line v <- M v.
template <int N, typename P>
__device__ __forceinline__ void gauss_sweep(P *buf, int total, int stride, const P *M, int t,
                                            int T) {
  const int lines = total / N;
  for (int l = t; l < lines; l += T) {
    const int lo = l % stride, hi = l / stride;
    P *p = buf + lo + hi * stride * N;
    P v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * stride];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      P s = M[q * N] * v[0];
#pragma unroll
      for (int m = 1; m < N; ++m) s += M[q * N + m] * v[m];
      p[q * stride] = s;
    }
  }
}

template <int D, int N, int DX, typename P>
__global__ void __launch_bounds__(gauss_threads(ipow(N, D)))
    stage_gauss_kernel(const StageParams<P> prm, const GaussTables<P> gt) {
  constexpr int ND = ipow(N, D), NF = ND / N, T = gauss_threads(ND), R = (ND + T - 1) / T;
  constexpr int NXN = ipow(N, DX);
  // With at most 16 nodes per thread the input solution and du stay in
  // registers from the start; larger cells read them again for the update.
  constexpr bool KEEP = R <= 16;
  extern __shared__ unsigned char smem_raw[];
  P *W = reinterpret_cast<P *>(smem_raw);  // the cell, then U, then Y and L(u)
  P *F = W + ND;                           // face layers [side][p]
  P *EG = F + 2 * NF;                      // E at the x-Gauss points [xq][comp]
  const int t = threadIdx.x;
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
  P *ducell = prm.du + (uint64_t)cell * ND;
  constexpr int RK = KEEP ? R : 1;
  double ud[RK];
  P dv[RK];
  if constexpr (KEEP) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = t + T * r;
      ud[r] = q < ND ? ucell[q] : 0.0;
    }
    if (stage && prm.read_du) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = t + T * r;
        dv[r] = q < ND ? ducell[q] : P(0);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = t + T * r;
      if (q < ND) W[q] = (P)ud[r];
    }
  } else {
    for (int q = t; q < ND; q += T) W[q] = (P)ucell[q];
  }
  if (phase) {
    // E at the x-Gauss points: the nodal interpolant of the cell's E table
    unsigned xcell = 0, xs = 1;
#pragma unroll
    for (int m = 0; m < DX; ++m) {
      xcell += c[m] * xs;
      xs *= prm.cells[m];
    }
    const P *e = prm.E + (uint64_t)xcell * NXN * DX;
    for (int idx = t; idx < NXN * DX; idx += T) {
      const int xq = idx / DX, comp = idx % DX;
      P s = P(0);
      for (int xn = 0; xn < NXN; ++xn) {
        P ph = P(1);
        int a = xq, b = xn;
#pragma unroll
        for (int m = 0; m < DX; ++m) {
          ph *= gt.B[(a % N) * N + (b % N)];
          a /= N;
          b /= N;
        }
        s += ph * e[xn * DX + comp];
      }
      EG[idx] = prm.esign * s;
    }
  }
  __syncthreads();
  // U = (B x ... x B) u
#pragma unroll
  for (int j = 0; j < D; ++j) {
    gauss_sweep<N>(W, ND, ipow(N, j), gt.B, t, T);
    __syncthreads();
  }

  // a_j at a Gauss point given by its digits (digit j itself is not used:
  // a_j does not depend on x_j).
  auto a_at = [&](int j, const int *dig) -> P {
    if (!phase) return prm.a_const[j];
    if (j < DX)
      return prm.vlo[DX + j] + (P(c[DX + j]) + gt.g[dig[DX + j]]) * prm.vh[DX + j];
    int xq = 0;
#pragma unroll
    for (int m = DX - 1; m >= 0; --m) xq = xq * N + dig[m];
    return EG[xq * DX + (j - DX)];
  };

  // volume: Y = - sum_j a_j / h_j Dg_j U
  P Y[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = t + T * r;
    Y[r] = P(0);
    if (q >= ND) continue;
    int dig[D];
    int rem = q;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      dig[m] = rem % N;
      rem /= N;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int stride = ipow(N, j);
      const int base = q - dig[j] * stride;
      P s = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) s += gt.Dg[dig[j] * N + m] * W[base + m * stride];
      Y[r] -= a_at(j, dig) * prm.inv_h[j] * s;
    }
  }

  // faces, one dimension at a time
#pragma unroll 1
  for (int j = 0; j < D; ++j) {
    const int sj = ipow(N, j);
    __syncthreads();  // F is free
    const double *ul = prm.u_in + (uint64_t)left[j] * ND;
    const double *ur = prm.u_in + (uint64_t)right[j] * ND;
    for (int idx = t; idx < 2 * NF; idx += T) {
      const int side = idx / NF, p = idx % NF;
      const int lo = p % sj, hi = p / sj;
      // side 0 (face xi_j = 0): the left neighbour's layer i_j = k;
      // side 1 (xi_j = 1): the right neighbour's layer i_j = 0
      const int node = lo + (side ? 0 : N - 1) * sj + hi * sj * N;
      F[idx] = (P)(side ? ur : ul)[node];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
      gauss_sweep<N>(F, 2 * NF, ipow(N, a), gt.B, t, T);
      __syncthreads();
    }
    // scaled jumps at the face Gauss points
    for (int idx = t; idx < 2 * NF; idx += T) {
      const int side = idx / NF, p = idx % NF;
      const int lo = p % sj, hi = p / sj;
      const int base = lo + hi * sj * N;
      int dig[D];
      int rem = base;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        dig[m] = rem % N;
        rem /= N;
      }
      P uo = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) uo += gt.ext[side][m] * W[base + m * sj];
      const P a = a_at(j, dig);
      const P an = side ? a : -a;
      F[idx] = (an < P(0) ? an : P(0)) * (uo - F[idx]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = t + T * r;
      if (q >= ND) continue;
      const int qj = (q / sj) % N;
      const int p = q % sj + (q / (sj * N)) * sj;
      Y[r] += prm.inv_h[j] * (gt.lift[0][qj] * F[p] + gt.lift[1][qj] * F[NF + p]);
    }
  }
  __syncthreads();  // every read of U is done
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = t + T * r;
    if (q < ND) W[q] = Y[r];
  }
  __syncthreads();
  // L(u) = (B^{-1} x ... x B^{-1}) Y
#pragma unroll
  for (int j = 0; j < D; ++j) {
    gauss_sweep<N>(W, ND, ipow(N, j), gt.Binv, t, T);
    __syncthreads();
  }

  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = t + T * r;
      if (q < ND) ocell[q] = W[q];
    }
    return;
  }
  double *uocell = prm.u_out + (uint64_t)cell * ND;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = t + T * r;
    if (q >= ND) continue;
    const P L = W[q];
    P dold;
    double uin;
    if constexpr (KEEP) {
      dold = dv[r];
      uin = ud[r];
    } else {
      dold = prm.read_du ? ducell[q] : P(0);
      uin = ucell[q];
    }
    const P dn = prm.read_du ? prm.rk_a * dold + prm.dt * L : prm.dt * L;
    if (prm.write_du) ducell[q] = dn;
    uocell[q] = uin + prm.rk_b * (double)dn;
  }
}

}  // namespace hd
