// Fused LSRK stage on mapped configuration cells (the tensor-product mapping
// of Sec. 3.1 / 3.3) with Gauss-Lobatto collocation, six dimensions (3 x +
// 3 v) at degree 3, in the thread layout of the collocation kernel of
// stage_k3.h: thread t = lane + 64 * wave owns the 16 nodes (i1, i2, i3) =
// lane bits, i4 = wave, (i5, i6) = register index s = i5 + 4 i6.
//
// The operator is the weak form with the contravariant flux a^ = |J| J^-1 a
// at the nodes (which are the quadrature points), per node i:
//   Y_i = sum_j sum_m Dw[i_j][m] (a^_j u)_{i_j -> m}
//         - sum over the faces through i of lift (a^ . n) u*,   L_i = Y_i / |J|,
// Dw = W^-1 D^T W the weak derivative along one dimension, lift = 1 / w_0 at
// the face's boundary node and u* the upwind value (own if a^ . n >= 0,
// else the neighbour's). a^ of an x-dimension is adj(J) v: it varies along
// the line and is applied before the sweep; a^ of a v-dimension is
// |J| E / h: constant along v, it factors out of the line. The v-cell volume
// scales every term and the division by |J| alike, so it is left out. The
// metric (adjugate and determinant at the x-nodes, adjugate rows at the
// x-face nodes) is read per lane from the x-cell's table. Exact up to
// rounding: the same operator as the sweep kernel of stage_gauss.h with
// collocation tables, and the oracle's mapped collocation mode.
#pragma once

#include "stage_gauss.h"
#include "stage_k3_gauss.h"

namespace hd {

template <typename P>
struct K3MappedTables {
  P Dw[16];  // Dw[q * 4 + m] = D[m][q] w_m / w_q, D[q][m] = l'_m(xi_q)
  P winv;    // 1 / w_0 = 1 / w_3
};

// LDS: the weak-derivative table (lane-indexed), the cell.
template <typename P>
constexpr size_t k3m_lds_bytes() {
  return (size_t)(16 + kK3Nodes) * sizeof(P);
}

template <typename P, int OPT>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(sizeof(P) == 8 ? 2 : 3, sizeof(P) == 8 ? 2 : 3)))
    stage_k3m_kernel(const StageParams<P> prm, const K3MappedTables<P> mt) {
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr int ND = kK3Nodes;
  constexpr int MXE = 10, NFX = 16;  // [xq][adj (3x3), det], then [j][side][face x-point][3]
  extern __shared__ __align__(16) unsigned char smem_raw[];
  P *tDw = reinterpret_cast<P *>(smem_raw);
  P *cellb = tDw + 16;
  const int t = threadIdx.x;
  const int l = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int i1 = l & 3, i2 = (l >> 2) & 3, i3 = l >> 4;

  unsigned cell = blockIdx.x;
  if (prm.xcd_remap) cell = xcd_tile(cell, prm.nblocks);
  unsigned c[6], left[6], right[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    c[j] = (cell / prm.cstride[j]) % prm.cells[j];
    const unsigned nj = prm.cells[j], st = prm.cstride[j];
    left[j] = c[j] == 0 ? cell + (nj - 1) * st : cell - st;
    right[j] = c[j] == nj - 1 ? cell - (nj - 1) * st : cell + st;
  }
  const unsigned xcell = c[0] + prm.cells[0] * (c[1] + prm.cells[1] * c[2]);
  const double *ucell = prm.u_in + (uint64_t)cell * ND;
  double ud[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) ud[s] = ucell[t + 256 * s];
  // metric at this lane's x-node
  const double *mg = prm.xmetric + (uint64_t)xcell * gauss_metric_elems(4, 3);
  P adj[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) adj[i] = (P)mg[l * MXE + i];
  const P det = (P)mg[l * MXE + 9];
  // field in the specialised kernel's form: a_{x_k} = vb_k + xi vh_k at the
  // velocity node, a_{v_j} = esign E_j at the lane's x-node
  const P *e = prm.E + ((uint64_t)xcell * 64 + l) * 3;
  P ev[3], vb[3], vhh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    ev[j] = prm.esign * e[j];
    vhh[j] = prm.vh[3 + j];
    vb[j] = prm.vlo[3 + j] + P(c[3 + j]) * vhh[j];
  }
  const P v1 = vb[0] + prm.xi[w] * vhh[0];  // velocity 1 at i4 = wave
  auto v2 = [&](int s) { return vb[1] + prm.xi[s & 3] * vhh[1]; };
  auto v3 = [&](int s) { return vb[2] + prm.xi[s >> 2] * vhh[2]; };

  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 16; ++q) tDw[q] = mt.Dw[q];
  }
  P u[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    u[s] = to_p<P>(ud[s]);
    cellb[t + 256 * s] = u[s];
  }
  __syncthreads();  // table and cell in LDS

  // ---- volume, v-dimensions: a^ = |J| E / h constant along the line ----
  const P av0 = det * prm.inv_h[3] * ev[0], av1 = det * prm.inv_h[4] * ev[1],
          av2 = det * prm.inv_h[5] * ev[2];
  P y[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int i5 = s & 3, i6 = s >> 2;
    P d4 = P(0), d5 = P(0), d6 = P(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      d4 += tDw[w * 4 + m] * cellb[l + 64 * m + 256 * s];
      d5 += mt.Dw[i5 * 4 + m] * u[4 * i6 + m];
      d6 += mt.Dw[i6 * 4 + m] * u[i5 + 4 * m];
    }
    y[s] = av0 * d4 + av1 * d5 + av2 * d6;
  }
  // ---- volume, x-dimensions: the sweep of a^_j u, a^_j = adj row j . v ----
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    P p[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
      p[s] = (adj[3 * j] * v1 + adj[3 * j + 1] * v2(s) + adj[3 * j + 2] * v3(s)) * u[s];
    if (j == 0) k3g_lane<1, 16>(tDw, p, l);
    else if (j == 1) k3g_lane<2, 16>(tDw, p, l);
    else k3g_lane<3, 16>(tDw, p, l);
#pragma unroll
    for (int s = 0; s < 16; ++s) y[s] += p[s];
  }

  // ---- faces: every side, - lift (a^ . n) u* at its boundary nodes ----
  const P winv = mt.winv;
  {
    // dim 5 (v_2): boundary nodes s = 4 q (i5 = 0, side 0) and 4 q + 3
    // (side 1); a^ is the same on both, so the neighbour layer of the one
    // inflow side is loaded: left i5 = 3 where a^ > 0, right i5 = 0 else.
    const double *un = prm.u_in + (uint64_t)(av1 > P(0) ? left[4] : right[4]) * ND;
    const int o = av1 > P(0) ? 3 : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const P nb = to_p<P>(un[t + 256 * (o + 4 * q)]);
      const P an0 = -av1, an1 = av1;
      y[4 * q] -= winv * an0 * (an0 >= P(0) ? u[4 * q] : nb);
      y[4 * q + 3] -= winv * an1 * (an1 >= P(0) ? u[4 * q + 3] : nb);
    }
  }
  {
    // dim 6 (v_3): boundary nodes s = q (i6 = 0) and q + 12 (i6 = 3)
    const double *un = prm.u_in + (uint64_t)(av2 > P(0) ? left[5] : right[5]) * ND;
    const int o = av2 > P(0) ? 12 : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const P nb = to_p<P>(un[t + 256 * (o + q)]);
      const P an0 = -av2, an1 = av2;
      y[q] -= winv * an0 * (an0 >= P(0) ? u[q] : nb);
      y[q + 12] -= winv * an1 * (an1 >= P(0) ? u[q + 12] : nb);
    }
  }
  if (w == 0 || w == 3) {
    // dim 4 (v_1): boundary nodes on waves 0 (side 0) and 3 (side 1)
    const bool s1 = w == 3;
    const P an = s1 ? av0 : -av0;
    const double *un = prm.u_in + (uint64_t)(s1 ? right[3] : left[3]) * ND;
    const int nl = s1 ? l : l + 192;  // the neighbour's node of the face
    if (an < P(0)) {
#pragma unroll
      for (int s = 0; s < 16; ++s) y[s] -= winv * an * to_p<P>(un[nl + 256 * s]);
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) y[s] -= winv * an * u[s];
    }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    // x-dimension j: boundary lanes (lane digit j = 0 or 3); a^ . n from
    // the face's adjugate row varies with the node, so does the side taken
    const int ij = j == 0 ? i1 : (j == 1 ? i2 : i3);
    if (ij == 0 || ij == 3) {
      const int side = ij == 3 ? 1 : 0;
      const int sj = 1 << (2 * j);
      const int xp = l % sj + (l / (sj * 4)) * sj;  // the face's x-point
      const double *mf = mg + 64 * MXE + ((j * 2 + side) * NFX + xp) * 3;
      const P f0 = (P)mf[0], f1 = (P)mf[1], f2 = (P)mf[2];
      const double *un = prm.u_in + (uint64_t)(side ? right[j] : left[j]) * ND;
      const int nl = side ? l - 3 * sj : l + 3 * sj;  // digit j: 3 <-> 0
      // FP32: whether any of the lane's 16 face nodes has inflow, from the
      // least of a^ . n over its (v2, v3) nodes, which separates over the
      // two components and sits at the cell's end nodes (6.8 against 7.1 ms
      // per stage at 8^6; FP64 measured 8.7 against 8.5 ms and loads always).
      const P g0 = side ? f0 : -f0, g1 = side ? f1 : -f1, g2 = side ? f2 : -f2;
      const P m2a = g1 * v2(0), m2b = g1 * v2(3), m3a = g2 * v3(0), m3b = g2 * v3(12);
      const bool need = sizeof(P) == 8 || g0 * v1 + (m2a < m2b ? m2a : m2b) + (m3a < m3b ? m3a : m3b) < P(0);
      // then the neighbour's 16 values in one batch of loads (a load per
      // inflow node, under its own condition, kept them in flight one at a
      // time: 10.6 against 7.1 ms per FP32 stage at 8^6)
      double nbv[16];
      if (need) {
#pragma unroll
        for (int s = 0; s < 16; ++s) nbv[s] = un[nl + 64 * w + 256 * s];
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const P a = f0 * v1 + f1 * v2(s) + f2 * v3(s);
        const P an = side ? a : -a;
        const P us = need && an < P(0) ? to_p<P>(nbv[s]) : u[s];
        y[s] -= winv * an * us;
      }
    }
  }
  const P rdet = P(1) / det;
#pragma unroll
  for (int s = 0; s < 16; ++s) y[s] *= rdet;

  // ---- output / RK update ----
  const bool stage = prm.mode == 1;
  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
#pragma unroll
    for (int s = 0; s < 16; ++s) ocell[t + 256 * s] = y[s];
    return;
  }
  P *ducell = prm.du + (uint64_t)cell * ND;
  P dv[16];
  if (prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.rk_a * ld_opt<NT>(ducell + t + 256 * s) + prm.dt * y[s];
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.dt * y[s];
  }
  if (prm.write_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) st_opt<NT>(ducell + t + 256 * s, dv[s]);
  }
  double *uocell = prm.u_out + (uint64_t)cell * ND;
#pragma unroll
  for (int s = 0; s < 16; ++s) st_opt<NT>(uocell + t + 256 * s, ud[s] + prm.rk_b * (double)dv[s]);
}

}  // namespace hd
