// Fused LSRK stage with Gauss-Legendre quadrature on mapped configuration
// cells (the tensor-product mapping of Sec. 3.1 / 3.3 with the quadrature of
// Sec. 2.5), six dimensions (3 x + 3 v) at degree 3, in the thread layout of
// the collocation kernel of stage_k3.h: thread t = lane + 64 * wave owns the
// 16 nodes (i1, i2, i3) = lane bits, i4 = wave, (i5, i6) = register index
// s = i5 + 4 i6.
//
// The operator is the weak form of the sweep kernel (stage_gauss.h, MAPPED):
// with U the values at the Gauss points and ahat = |J| J^-1 a,
//   L(u) = B^-1 [ (sum_j Dw_j (ahat_j U) - sum_faces lift_s (ahat.n) u*) / |J| ],
// Dw[q][m] = Dg[m][q] om_m / om_q the weak derivative along one dimension.
// It is evaluated with the x-dimensions at their Gauss points and the
// v-dimensions in nodal form (the accumulator Z holds B^-1 along v of the
// bracket), which spares every velocity transform but those of the x-face
// jumps:
//  - the mapping deforms x only, so ahat_x = adj(A) v is linear in v, and
//    multiplication by v_c at the Gauss points is, in nodal form, the matrix
//    alpha_c I + vh_c G along v_c (G = B^-1 diag(g) B). The x-volume term is
//    Dw along x_j of sum_c adj_jc V_c with V_c = (alpha_c I + vh_c G_c) Ux,
//    Ux = B(x3) u; the own traces of the x-faces are lift_s ext_s of
//    sum_c f_c V_c, f the adjugate row of the face point;
//  - ahat_v / |J| = E / h_v depends on x only: the v-terms are those of the
//    Cartesian cells (stage_k3_gauss.h), the volume in strong form (exact
//    along v, where ahat is constant) and the upwind jumps of the v-faces;
//  - at an x-face with inflow points, the jump of the neighbour's trace
//    against the own one is carried to the face's Gauss points in all five
//    tangential dimensions, weighted with min(ahat.n, 0) point by point and
//    returned to nodal form along v; each wave takes one face's layer whole.
//    (Applying ahat.n in nodal form where a whole face has inflow, like the
//    volume term, measured slower.)
// The division by |J| acts on the x-terms only (the v-terms are scaled by
// |J| before they enter Z). Exact up to rounding: the same operator as the
// sweep kernel's mapped Gauss-Legendre mode and the oracle's mapped
// Gauss-Legendre mode.
#pragma once

#include "stage_gauss.h"
#include "stage_k3_gauss.h"

namespace hd {

template <typename P>
struct K3MGaussTables {
  P B[16];        // B[q * 4 + i] = l_i(g_q)
  P Binv[16];     // B^-1
  P Dt[16];       // B^-1 Dg B: the derivative in nodal form
  P G[16];        // B^-1 diag(g) B: multiplication by the Gauss coordinate
  P Dw[16];       // Dw[q * 4 + m] = Dg[m][q] om_m / om_q
  P Blift[2][4];  // B^-1 lift_s: a face value lifted in nodal form
  P ext[2][4];    // ext[s][q]: the trace at xi = s from the Gauss values
  P lift[2][4];   // lift[s][q] = ext[s][q] / om_q
  P g[4];         // Gauss points on [0, 1]
};

// LDS: the lane-indexed tables, the cell (nodal), Ux, one face layer.
constexpr int kK3mgTab = 112;
template <typename P>
constexpr size_t k3mg_lds_bytes() {
  return (size_t)(kK3mgTab + 2 * kK3Nodes + kK3Face) * sizeof(P);
}

// 4 x 4 matrix M (row-major, kernel argument) along i5 and along i6, the
// register digits: out(i) = sum_m M[i][m] in(m).
template <typename P>
__device__ __forceinline__ void k3mg_reg5(const P (&M)[16], P (&v)[16]) {
#pragma unroll
  for (int i6 = 0; i6 < 4; ++i6) {
    const P a0 = v[4 * i6], a1 = v[4 * i6 + 1], a2 = v[4 * i6 + 2], a3 = v[4 * i6 + 3];
#pragma unroll
    for (int i5 = 0; i5 < 4; ++i5)
      v[i5 + 4 * i6] = M[i5 * 4] * a0 + M[i5 * 4 + 1] * a1 + M[i5 * 4 + 2] * a2 + M[i5 * 4 + 3] * a3;
  }
}
template <typename P>
__device__ __forceinline__ void k3mg_reg6(const P (&M)[16], P (&v)[16]) {
#pragma unroll
  for (int i5 = 0; i5 < 4; ++i5) {
    const P a0 = v[i5], a1 = v[i5 + 4], a2 = v[i5 + 8], a3 = v[i5 + 12];
#pragma unroll
    for (int i6 = 0; i6 < 4; ++i6)
      v[i5 + 4 * i6] = M[i6 * 4] * a0 + M[i6 * 4 + 1] * a1 + M[i6 * 4 + 2] * a2 + M[i6 * 4 + 3] * a3;
  }
}

// Sum over the four lanes of a line along lane dimension LD (1, 2, 3); the
// sum lands on all four.
template <int LD, typename P>
__device__ __forceinline__ P k3mg_line_sum(P x) {
  if constexpr (LD == 1) {
    x += dpp_move<0xB1>(x);  // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);  // quad_perm [2, 3, 0, 1]
  } else if constexpr (LD == 2) {
    x += dpp_move<row_ror(8)>(x);
    x += dpp_move<row_ror(4)>(x);
  } else {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
  }
  return x;
}

// Two workgroups per CU in both precisions (FP64: the LDS; the FP64 kernel
// spills some values, still faster than one workgroup without spills; FP32
// without spills, faster than three with them: 14.6 against 15.9 ms per
// stage at 8^6).
template <typename P, int OPT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
    stage_k3mg_kernel(const StageParams<P> prm, const K3MGaussTables<P> mt) {
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr int ND = kK3Nodes;
  constexpr int MXE = 10, NFX = 16;  // metric: [xq][adj (3x3), det], then [j][side][face x-point][3]
  extern __shared__ __align__(16) unsigned char smem_raw[];
  P *tB = reinterpret_cast<P *>(smem_raw);
  P *tBinv = tB + 16, *tDt = tB + 32, *tG = tB + 48, *tDw = tB + 64, *tBl = tB + 80;
  P *tExt = tB + 88, *tLift = tB + 96, *tg = tB + 104;
  P *cellb = tB + kK3mgTab;  // u (nodal)
  P *uxb = cellb + ND;       // Ux = B(x3) u
  P *faceb = uxb + ND;       // one face layer
  __shared__ int fmask;      // sides with inflow points: bit 2 j + side
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
  // metric at this lane's x-Gauss point
  const double *mg = prm.xmetric + (uint64_t)xcell * gauss_metric_elems(4, 3);
  const P det = (P)mg[l * MXE + 9];
  // field in the specialised kernel's form: v_c = alpha_c + vh_c g at the
  // velocity Gauss coordinate g; a_{v_j} = esign E_j, here at the x-nodes
  const P *e = prm.E + ((uint64_t)xcell * 64 + l) * 3;
  P eg[3], alpha[3], vhh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    eg[j] = prm.esign * e[j];
    vhh[j] = prm.vh[3 + j];
    alpha[j] = prm.vlo[3 + j] + P(c[3 + j]) * vhh[j];
  }
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      tB[q] = mt.B[q];
      tBinv[q] = mt.Binv[q];
      tDt[q] = mt.Dt[q];
      tG[q] = mt.G[q];
      tDw[q] = mt.Dw[q];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        tBl[4 * sd + i] = mt.Blift[sd][i];
        tExt[4 * sd + i] = mt.ext[sd][i];
        tLift[4 * sd + i] = mt.lift[sd][i];
      }
      tg[i] = mt.g[i];
    }
    fmask = 0;
  }
  __syncthreads();  // tables, mask cleared
  // E at this lane's x-Gauss point (the nodal interpolant)
  k3g_x3<3>(tB, eg, l);

  // Inflow sides (bit 2 j + side). v-faces: from the sign of E at the
  // x-Gauss points. x-face (j, side): the least of ahat.n = n_s f . v over
  // the velocity Gauss grid, which separates over the components (linear in
  // each v_c); f is the adjugate row at this lane's tangential x-point.
  {
    int mine = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      mine |= (eg[j] > P(0) ? 1 : 0) << (6 + 2 * j);
      mine |= (eg[j] < P(0) ? 1 : 0) << (7 + 2 * j);
      const int sj = 1 << (2 * j);
      const int xp = l % sj + (l / (sj * 4)) * sj;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const double *mf = mg + 64 * MXE + ((j * 2 + sd) * NFX + xp) * 3;
        P mn = P(0);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          const P f = sd ? (P)mf[cc] : -(P)mf[cc];
          const P lo = f * (alpha[cc] + vhh[cc] * mt.g[0]), hi = f * (alpha[cc] + vhh[cc] * mt.g[3]);
          mn += lo < hi ? lo : hi;
        }
        mine |= (mn < P(0) ? 1 : 0) << (2 * j + sd);
      }
    }
    if (mine) atomicOr(&fmask, mine);
  }

  // the cell to LDS; Ux to registers and LDS
  P ux[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    ux[s] = to_p<P>(ud[s]);
    cellb[t + 256 * s] = ux[s];
  }
  k3g_x3<16>(tB, ux, l);
#pragma unroll
  for (int s = 0; s < 16; ++s) uxb[t + 256 * s] = ux[s];
  __syncthreads();  // cell, Ux, mask
  const int active = fmask;

  // ---- volume, v-dimensions (strong form), scaled by |J|; from the same
  // values along i4, V1 = (alpha_1 I + vh_1 G) Ux along i4 ----
  P z[16], V1[16];
  {
    const P c4 = det * prm.inv_h[3] * eg[0], c5 = det * prm.inv_h[4] * eg[1],
            c6 = det * prm.inv_h[5] * eg[2];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i5 = s & 3, i6 = s >> 2;
      P d4 = P(0), d5 = P(0), d6 = P(0), g1 = P(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const P x = uxb[l + 64 * m + 256 * s];
        d4 += tDt[w * 4 + m] * x;
        g1 += tG[w * 4 + m] * x;
        d5 += mt.Dt[i5 * 4 + m] * ux[4 * i6 + m];
        d6 += mt.Dt[i6 * 4 + m] * ux[i5 + 4 * m];
      }
      z[s] = -(c4 * d4 + c5 * d5 + c6 * d6);
      V1[s] = alpha[0] * ux[s] + vhh[0] * g1;
    }
  }

  // V1 to LDS in place of Ux (every wave has read Ux along i4): the
  // registers stay free for the x-passes, which read back their own values.
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 16; ++s) uxb[t + 256 * s] = V1[s];
  asm volatile("" ::: "memory");

  // ---- x-dimensions: weak volume term and the own traces of both faces ----
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int sj = 1 << (2 * j);
    const int xp = l % sj + (l / (sj * 4)) * sj;
    const int ij = j == 0 ? i1 : (j == 1 ? i2 : i3);
    const double *mf0 = mg + 64 * MXE + ((j * 2) * NFX + xp) * 3;
    const double *mf1 = mf0 + NFX * 3;
    const P f00 = (P)mf0[0], f01 = (P)mf0[1], f02 = (P)mf0[2];
    const P f10 = (P)mf1[0], f11 = (P)mf1[1], f12 = (P)mf1[2];
    const P a0 = (P)mg[l * MXE + 3 * j], a1 = (P)mg[l * MXE + 3 * j + 1], a2 = (P)mg[l * MXE + 3 * j + 2];
    const P e0 = tExt[ij], e1 = tExt[4 + ij], lf0 = tLift[ij], lf1 = tLift[4 + ij];
    // Four register values at a time (the lane transform acts on each value
    // by itself): only four volume terms are live beside z and Ux.
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
    P p[4];
#pragma unroll
    for (int si = 0; si < 4; ++si) {
      const int s = 4 * c4 + si;
      const int i5 = s & 3, i6 = s >> 2;
      P g2 = P(0), g3 = P(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        g2 += mt.G[i5 * 4 + m] * ux[4 * i6 + m];
        g3 += mt.G[i6 * 4 + m] * ux[i5 + 4 * m];
      }
      const P V1s = uxb[t + 256 * s];
      const P V2 = alpha[1] * ux[s] + vhh[1] * g2;
      const P V3 = alpha[2] * ux[s] + vhh[2] * g3;
      p[si] = a0 * V1s + a1 * V2 + a2 * V3;
      P w0 = e0 * (f00 * V1s + f01 * V2 + f02 * V3);
      P w1 = e1 * (f10 * V1s + f11 * V2 + f12 * V3);
      if (j == 0) {
        w0 = k3mg_line_sum<1>(w0);
        w1 = k3mg_line_sum<1>(w1);
      } else if (j == 1) {
        w0 = k3mg_line_sum<2>(w0);
        w1 = k3mg_line_sum<2>(w1);
      } else {
        w0 = k3mg_line_sum<3>(w0);
        w1 = k3mg_line_sum<3>(w1);
      }
      // - lift_s (ahat.n) u_own, n_0 = -1, n_1 = +1
      z[s] += lf0 * w0 - lf1 * w1;
    }
    if (j == 0) k3g_lane<1, 4>(tDw, p, l);
    else if (j == 1) k3g_lane<2, 4>(tDw, p, l);
    else k3g_lane<3, 4>(tDw, p, l);
#pragma unroll
    for (int si = 0; si < 4; ++si) z[4 * c4 + si] += p[si];
    }
  }

  // ---- faces of the v-dimensions: upwind jumps (Cartesian form), scaled by |J| ----
#pragma unroll
  for (int j = 3; j < 6; ++j) {
#pragma unroll 1
    for (int sd = 0; sd < 2; ++sd) {
      if (!((active >> (2 * j + sd)) & 1)) continue;
      // face node p = t + 256 q: the own-minus-neighbour nodal jump
      const double *un = prm.u_in + (uint64_t)(sd ? right[j] : left[j]) * ND;
      P f[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int node0 = k3_face_node0(t + 256 * q, j);
        const int far = node0 + 3 * (1 << (2 * j));
        f[q] = cellb[sd ? far : node0] - to_p<P>(un[sd ? node0 : far]);
      }
      k3g_x3<4>(tB, f, l);
      const P a = sd ? eg[j - 3] : -eg[j - 3];
      const P sc = det * prm.inv_h[j] * (a < P(0) ? a : P(0));
#pragma unroll
      for (int q = 0; q < 4; ++q) f[q] *= sc;
      const P *bl = tBl + 4 * sd;
      if (j == 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i5 = 0; i5 < 4; ++i5) z[i5 + 4 * q] += bl[i5] * f[q];
      } else if (j == 5) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i6 = 0; i6 < 4; ++i6) z[q + 4 * i6] += bl[i6] * f[q];
      } else {
        // along i4 = wave: face point (lane, i5 = wave, i6 = q) via LDS
        __syncthreads();  // earlier readers of the face buffer are done
#pragma unroll
        for (int q = 0; q < 4; ++q) faceb[t + 256 * q] = f[q];
        __syncthreads();
        const P wl = bl[w];
#pragma unroll
        for (int s = 0; s < 16; ++s) z[s] += wl * faceb[l + 64 * s];
      }
    }
  }

  // ---- x-faces with inflow points: min(ahat.n, 0) (u_nbr - u_own) ----
  // Rounds of up to four active faces. Face point p = t + 256 q of x-face j
  // has the digits (tangential x, i4, i5, i6) = p, so the workgroup writes
  // the nodal jumps of a face into a 1024-value slot (the buffer of V1,
  // free now); wave k then holds slot k whole, 64 lanes (tangential x, i4)
  // by 16 registers (i5, i6), carries it to the Gauss points in all five
  // dimensions with lane and register transforms, weights it with
  // min(ahat.n, 0) and returns it to nodal form along v; every thread then
  // lifts its line's values along x_j.
  int pending = active & 63;
#pragma unroll 1
  while (pending) {
    int round = 0, cnt = 0;
    {
      int r = pending;
      while (r && cnt < 4) {
        round |= r & -r;
        r &= r - 1;
        ++cnt;
      }
    }
    pending &= ~round;
    // the neighbour layers of the round's faces, all loads in flight at once
    double nb[6][4];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (!((round >> f) & 1)) continue;
      const int j = f >> 1, sd = f & 1;
      const unsigned nbr = sd ? right[j] : left[j];
      const double *un = prm.u_in + (uint64_t)nbr * ND;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int node0 = k3_face_node0(t + 256 * q, j);
        nb[f][q] = un[sd ? node0 : node0 + 3 * (1 << (2 * j))];
      }
    }
    __syncthreads();  // earlier readers of the slots are done
    {
      P *slot = uxb;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!((round >> f) & 1)) continue;
        const int j = f >> 1, sd = f & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int node0 = k3_face_node0(t + 256 * q, j);
          slot[t + 256 * q] = to_p<P>(nb[f][q]) - cellb[sd ? node0 + 3 * (1 << (2 * j)) : node0];
        }
        slot += kK3Face;
      }
    }
    __syncthreads();
    if (w < cnt) {
      // this wave's face: the w-th of the round
      int r = round;
      for (int i = 0; i < w; ++i) r &= r - 1;
      const int f = __builtin_ctz(r), sd = f & 1;
      P *slot = uxb + kK3Face * w;
      P jv[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) jv[s] = slot[l + 64 * s];
      k3g_lane<1, 16>(tB, jv, l);  // tangential x (lower dimension)
      k3g_lane<2, 16>(tB, jv, l);  // tangential x (upper dimension)
      k3g_lane<3, 16>(tB, jv, l);  // i4
      k3mg_reg5(mt.B, jv);
      k3mg_reg6(mt.B, jv);
      const double *mf = mg + 64 * MXE + (f * NFX + (l & 15)) * 3;
      const P fa = sd ? (P)mf[0] : -(P)mf[0], fb = sd ? (P)mf[1] : -(P)mf[1],
              fc = sd ? (P)mf[2] : -(P)mf[2];
      const P v1 = alpha[0] + vhh[0] * tg[l >> 4];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int i5 = s & 3, i6 = s >> 2;
        const P an = fa * v1 + fb * (alpha[1] + vhh[1] * mt.g[i5]) + fc * (alpha[2] + vhh[2] * mt.g[i6]);
        jv[s] *= an < P(0) ? an : P(0);
      }
      k3g_lane<3, 16>(tBinv, jv, l);
      k3mg_reg5(mt.Binv, jv);
      k3mg_reg6(mt.Binv, jv);
#pragma unroll
      for (int s = 0; s < 16; ++s) slot[l + 64 * s] = jv[s];
    }
    __syncthreads();
    // lift along x_j: - lift_s[q_j] F at the line's face point
    {
      const P *slot = uxb;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!((round >> f) & 1)) continue;
        const int j = f >> 1, sd = f & 1, sj = 1 << (2 * j);
        const int ij = (l >> (2 * j)) & 3;
        const int tl = l % sj + (l / (sj * 4)) * sj;
        const P lq = tLift[4 * sd + ij];
#pragma unroll
        for (int s = 0; s < 16; ++s) z[s] -= lq * slot[tl + 16 * w + 64 * s];
        slot += kK3Face;
      }
    }
  }

  // ---- division by |J|, back to the x-nodes ----
  const P rdet = P(1) / det;
#pragma unroll
  for (int s = 0; s < 16; ++s) z[s] *= rdet;
  k3g_lane<3, 16>(tBinv, z, l);
  k3g_lane<2, 16>(tBinv, z, l);
  k3g_lane<1, 16>(tBinv, z, l);

  // ---- output / RK update ----
  const bool stage = prm.mode == 1;
  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
#pragma unroll
    for (int s = 0; s < 16; ++s) ocell[t + 256 * s] = z[s];
    return;
  }
  P *ducell = prm.du + (uint64_t)cell * ND;
  P dv[16];
  if (prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.rk_a * ld_opt<NT>(ducell + t + 256 * s) + prm.dt * z[s];
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.dt * z[s];
  }
  if (prm.write_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) st_opt<NT>(ducell + t + 256 * s, dv[s]);
  }
  double *uocell = prm.u_out + (uint64_t)cell * ND;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    double uo;
    if constexpr (sizeof(P) == sizeof(double)) uo = (double)cellb[t + 256 * s];
    else uo = ucell[t + 256 * s];
    st_opt<NT>(uocell + t + 256 * s, uo + prm.rk_b * (double)dv[s]);
  }
}

}  // namespace hd
