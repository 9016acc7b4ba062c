// Fused LSRK stage with Gauss-Legendre quadrature (k+1 points per
// dimension) for six dimensions (3 x + 3 v) at degree 3, on Cartesian cells,
// in the thread layout of the collocation kernel of stage_k3.h: thread
// t = lane + 64 * wave owns the 16 nodes (i1, i2, i3) = lane bits, i4 = wave,
// (i5, i6) = register index s = i5 + 4 i6.
//
// The operator is the Gauss-quadrature weak form of Sec. 2.5: with U the
// values at the Gauss points (U = B u per dimension, B[q][i] = l_i(g_q)),
//   L(u) = B^-1 [ -sum_j (a_j / h_j) Dg_j U + sum_faces lift_s (x) m (B u_jump) ]
// per cell, m = min(a.n, 0) the upwind weight at the face's Gauss points
// and lift_s the lifting of a face value into the Gauss points along j.
// Because B^-1 (x) ... (x) B^-1 undoes the transforms of every dimension on
// which a factor does not act, the operator is evaluated in nodal space
// with 4 x 4 matrices instead of transforms of the whole cell:
//  - x-dimension j: a_j = v_j depends on the velocity coordinate v_j only,
//    so the term is (alpha_j I + vh_j G) along v_j times Dt along x_j, with
//    Dt = B^-1 Dg B, G = B^-1 diag(g) B and v_j(g_q) = alpha_j + vh_j g_q;
//  - v-dimension j: a_j = E_j(x) at the x-Gauss points, so the term is
//    B^-1(x3) [E_j(g) * B(x3) (Dt along v_j) u] over the three x dimensions,
//    which are this layout's lane dimensions (DPP and lane shuffles);
//  - face of an x-dimension: (B^-1 lift_s) along x_j times
//    B^-1 diag(m(g)) B along v_j applied to the nodal jump of the face layer;
//  - face of a v-dimension: (B^-1 lift_s) along v_j times the x-transform
//    B^-1(x3) [m(g) * B(x3) jump].
// All of this is exact up to rounding: the same operator as the sweep
// kernel of stage_gauss.h and the oracle's Gauss mode.
#pragma once

#include "stage_k3.h"

namespace hd {

// 1D matrices of the Gauss-Legendre form at degree 3, row-major [i * 4 + m].
template <typename P>
struct K3GaussTables {
  P B[16];        // B[q * 4 + i] = l_i(g_q): nodal values to Gauss-point values
  P Binv[16];     // B^-1
  P Dt[16];       // B^-1 Dg B: the derivative along one dimension
  P G[16];        // B^-1 diag(g) B: multiplication by the Gauss coordinate
  P Blift[2][4];  // B^-1 lift_s: a face value lifted along its dimension
  P g[4];         // Gauss points on [0, 1]
};

// LDS: the lane-indexed tables (B, B^-1, Dt, G, the two lifts), the cell,
// four face layers.
constexpr int kK3gTab = 72;
template <typename P>
constexpr size_t k3g_lds_bytes() {
  return (size_t)(kK3gTab + kK3Nodes + 4 * kK3Face) * sizeof(P);
}

// Apply the 4 x 4 LDS table M (row-major) along lane dimension LD (1, 2, 3)
// to each of the NV values of every lane: out(i) = sum_m M[i][m] in(m), the
// index i being the lane's digit LD.
template <int LD, int NV, typename P>
__device__ __forceinline__ void k3g_lane(const P *M, P (&v)[NV], int l) {
  if constexpr (LD == 1) {
    const int i = l & 3;
    const P r0 = M[i * 4], r1 = M[i * 4 + 1], r2 = M[i * 4 + 2], r3 = M[i * 4 + 3];
#pragma unroll
    for (int s = 0; s < NV; ++s)
      v[s] = r0 * dpp_move<quad_bcast(0)>(v[s]) + r1 * dpp_move<quad_bcast(1)>(v[s]) +
             r2 * dpp_move<quad_bcast(2)>(v[s]) + r3 * dpp_move<quad_bcast(3)>(v[s]);
  } else if constexpr (LD == 2) {
    // row rotation by 4n brings the lane with digit i - n
    const int i = (l >> 2) & 3;
    const P r0 = M[i * 4 + i], r1 = M[i * 4 + ((i - 1) & 3)], r2 = M[i * 4 + ((i - 2) & 3)],
            r3 = M[i * 4 + ((i - 3) & 3)];
#pragma unroll
    for (int s = 0; s < NV; ++s)
      v[s] = r0 * v[s] + r1 * dpp_move<row_ror(4)>(v[s]) + r2 * dpp_move<row_ror(8)>(v[s]) +
             r3 * dpp_move<row_ror(12)>(v[s]);
  } else {
    // lanes 16 apart: shuffles within the wave
    const int i = l >> 4, b = l & 15;
    const P r0 = M[i * 4], r1 = M[i * 4 + 1], r2 = M[i * 4 + 2], r3 = M[i * 4 + 3];
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const P x0 = __shfl(v[s], b, 64), x1 = __shfl(v[s], b + 16, 64);
      const P x2 = __shfl(v[s], b + 32, 64), x3 = __shfl(v[s], b + 48, 64);
      v[s] = r0 * x0 + r1 * x1 + r2 * x2 + r3 * x3;
    }
  }
}

// The transform along all three x (lane) dimensions.
template <int NV, typename P>
__device__ __forceinline__ void k3g_x3(const P *M, P (&v)[NV], int l) {
  k3g_lane<1, NV>(M, v, l);
  k3g_lane<2, NV>(M, v, l);
  k3g_lane<3, NV>(M, v, l);
}

// FP64: 2 waves per SIMD (256 VGPRs); FP32: 3 (168 VGPRs, a few values spilled,
// measured faster than 2 waves without spills).
template <typename P, int OPT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(P) == 8 ? 2 : 3, sizeof(P) == 8 ? 2 : 3)))
    stage_k3g_kernel(const StageParams<P> prm, const K3GaussTables<P> gt) {
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr int ND = kK3Nodes, F = kK3Face;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  P *tB = reinterpret_cast<P *>(smem_raw);
  P *tBinv = tB + 16, *tDt = tB + 32, *tG = tB + 48, *tBl = tB + 64;
  P *cellb = tB + kK3gTab;
  P *faceb = cellb + ND;  // four layers of F values
  __shared__ int vmask;   // inflow sides of the v-dimension faces
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
  // Field in the specialised kernel's form (stage_k3.h): a_{x_j} = alpha_j +
  // vh_j g at velocity Gauss coordinate g; a_{v_j} = esign E_j at the x-nodes.
  const unsigned xcell = c[0] + prm.cells[0] * (c[1] + prm.cells[1] * c[2]);
  const P *e = prm.E + ((uint64_t)xcell * 64 + l) * 3;
  P eg[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) eg[j] = prm.esign * e[j];
  P alpha[3], vhh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    vhh[j] = prm.vh[3 + j];
    alpha[j] = prm.vlo[3 + j] + P(c[3 + j]) * vhh[j];
  }
  // the cell's own values (raw FP64)
  const double *ucell = prm.u_in + (uint64_t)cell * ND;
  double ud[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) ud[s] = ucell[t + 256 * s];

  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      tB[q] = gt.B[q];
      tBinv[q] = gt.Binv[q];
      tDt[q] = gt.Dt[q];
      tG[q] = gt.G[q];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tBl[i] = gt.Blift[0][i];
      tBl[4 + i] = gt.Blift[1][i];
    }
    vmask = 0;
  }
  __syncthreads();  // tables, mask cleared
  // E at this lane's x-Gauss point
  k3g_x3<3>(tB, eg, l);
  // Inflow sides. x-dimension j (uniform): side 0 (face xi_j = 0, normal -1)
  // where some a(g_q) > 0, side 1 where some a(g_q) < 0. v-dimensions: from
  // the signs of E at the x-Gauss points over the workgroup.
  int xmask = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const P a = alpha[j] + gt.g[q] * vhh[j];
      xmask |= (a > P(0) ? 1 : 0) << (2 * j);
      xmask |= (a < P(0) ? 1 : 0) << (2 * j + 1);
    }
  {
    int mine = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      mine |= (eg[j] > P(0) ? 1 : 0) << (2 * j);
      mine |= (eg[j] < P(0) ? 1 : 0) << (2 * j + 1);
    }
    if (mine) atomicOr(&vmask, mine);
  }
  __syncthreads();
  const int active = xmask | (vmask << 6);  // bit 2 j + side
  // Per dimension the first active side is taken in the first pass (its layer
  // loaded now), a second active side in a second pass.
  int prim[6], sec[6];
  bool any_sec = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const bool s0 = (active >> (2 * j)) & 1, s1 = (active >> (2 * j + 1)) & 1;
    prim[j] = s0 ? 0 : (s1 ? 1 : -1);
    sec[j] = s0 && s1 ? 1 : -1;
    any_sec |= s0 && s1;
  }
  double fv[6][4];
  auto load_layers = [&](const int(&side)[6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (side[j] < 0) continue;
      const double *un = prm.u_in + (uint64_t)(side[j] ? right[j] : left[j]) * ND;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int node0 = k3_face_node0(t + 256 * q, j);
        fv[j][q] = un[side[j] ? node0 : node0 + 3 * (1 << (2 * j))];
      }
    }
  };
  load_layers(prim);

  P u[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    u[s] = to_p<P>(ud[s]);
    cellb[t + 256 * s] = u[s];
  }
  __syncthreads();  // the cell in LDS

  P acc[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) acc[s] = P(0);
  // FP64: the v-face jumps stay at the x-Gauss points, lifted along v_j
  // (which commutes with the x-transforms) into zv, which joins the v-volume
  // terms before their one inverse x-transform (12.5 against 13.8 ms per
  // stage at 8^6, and no spills). FP32 transforms each jump back and lifts
  // it in nodal form: at its three waves per SIMD the extra live zv spills
  // (11.7 against 10.5 ms).
  constexpr bool kMergeV = sizeof(P) == sizeof(double);
  P zv[kMergeV ? 16 : 1];
#pragma unroll
  for (int s = 0; s < (kMergeV ? 16 : 1); ++s) zv[s] = P(0);

  // ---- faces ----
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    int side[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) side[j] = pass == 0 ? prim[j] : sec[j];
    if (pass == 1) {
      if (!any_sec) break;
      load_layers(side);
      __syncthreads();  // the first pass's layers are consumed
    }
    // Per dimension: the nodal jump own - neighbour on the face layer (face
    // node p = t + 256 q). x-dimensions: to LDS, weighted along v_j below.
    // v-dimensions: x-transform, upwind weight at the x-Gauss point, inverse
    // transform; dims 5 and 6 lift in registers, dim 4 via LDS.
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (side[j] < 0) continue;
      P f[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int node0 = k3_face_node0(t + 256 * q, j);
        P own;
        if (j == 4) own = side[j] ? u[3 + 4 * q] : u[4 * q];
        else if (j == 5) own = side[j] ? u[q + 12] : u[q];
        else own = cellb[side[j] ? node0 + 3 * (1 << (2 * j)) : node0];
        f[q] = own - to_p<P>(fv[j][q]);
      }
      if (j < 3) {
#pragma unroll
        for (int q = 0; q < 4; ++q) faceb[j * F + t + 256 * q] = f[q];
        continue;
      }
      k3g_x3<4>(tB, f, l);
      const P a = side[j] ? eg[j - 3] : -eg[j - 3];
      const P m = a < P(0) ? a : P(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) f[q] *= m;
      if constexpr (!kMergeV) {
        k3g_lane<3, 4>(tBinv, f, l);
        k3g_lane<2, 4>(tBinv, f, l);
        k3g_lane<1, 4>(tBinv, f, l);
      }
      const P ih = prm.inv_h[j];
      const P *bl = tBl + 4 * side[j];
      if (j == 3) {
#pragma unroll
        for (int q = 0; q < 4; ++q) faceb[3 * F + t + 256 * q] = f[q];
      } else if (j == 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i5 = 0; i5 < 4; ++i5) {
            if constexpr (kMergeV) zv[i5 + 4 * q] -= ih * bl[i5] * f[q];
            else acc[i5 + 4 * q] += ih * bl[i5] * f[q];
          }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i6 = 0; i6 < 4; ++i6) {
            if constexpr (kMergeV) zv[q + 4 * i6] -= ih * bl[i6] * f[q];
            else acc[q + 4 * i6] += ih * bl[i6] * f[q];
          }
      }
    }
    __syncthreads();
    // dim 4 face: lift along the waves
    if (side[3] >= 0) {
      const P wl = prm.inv_h[3] * tBl[4 * side[3] + w];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if constexpr (kMergeV) zv[s] -= wl * faceb[3 * F + l + 64 * s];
        else acc[s] += wl * faceb[3 * F + l + 64 * s];
      }
    }
    // x faces: Am = B^-1 diag(min(a(g) n, 0)) B along v_j, lifted along x_j
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (side[j] < 0) continue;
      P mq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const P a0 = alpha[j] + gt.g[q] * vhh[j];
        const P a = side[j] ? a0 : -a0;
        mq[q] = a < P(0) ? a : P(0);
      }
      const int ij = j == 0 ? i1 : (j == 1 ? i2 : i3);
      const P wl = prm.inv_h[j] * tBl[4 * side[j] + ij];
      if (j == 0) {
        // along v_1 = i4 = wave: the row of this wave
        P am[4];
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          P sum = P(0);
#pragma unroll
          for (int q = 0; q < 4; ++q) sum += tBinv[w * 4 + q] * mq[q] * gt.B[q * 4 + mm];
          am[mm] = sum;
        }
        const int pb = i2 + 4 * i3;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          P f = P(0);
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) f += am[mm] * faceb[pb + 16 * mm + 64 * s];
          acc[s] += wl * f;
        }
      } else {
        P am[16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) {
            P sum = P(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) sum += gt.Binv[i * 4 + q] * mq[q] * gt.B[q * 4 + mm];
            am[i * 4 + mm] = sum;
          }
        if (j == 1) {
          // along v_2 = i5; face index i1 + 4 i3 + 16 i4 + 64 i5 + 256 i6
          const int pb = F + i1 + 4 * i3 + 16 * w;
#pragma unroll
          for (int i6 = 0; i6 < 4; ++i6) {
            P jv[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) jv[mm] = faceb[pb + 64 * mm + 256 * i6];
#pragma unroll
            for (int i5 = 0; i5 < 4; ++i5) {
              P f = P(0);
#pragma unroll
              for (int mm = 0; mm < 4; ++mm) f += am[i5 * 4 + mm] * jv[mm];
              acc[i5 + 4 * i6] += wl * f;
            }
          }
        } else {
          // along v_3 = i6; face index i1 + 4 i2 + 16 i4 + 64 i5 + 256 i6
          const int pb = 2 * F + i1 + 4 * i2 + 16 * w;
#pragma unroll
          for (int i5 = 0; i5 < 4; ++i5) {
            P jv[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) jv[mm] = faceb[pb + 64 * i5 + 256 * mm];
#pragma unroll
            for (int i6 = 0; i6 < 4; ++i6) {
              P f = P(0);
#pragma unroll
              for (int mm = 0; mm < 4; ++mm) f += am[i6 * 4 + mm] * jv[mm];
              acc[i5 + 4 * i6] += wl * f;
            }
          }
        }
      }
    }
  }

  const int off3 = (l & 15) + 64 * w;  // the lane's line along i3 in the cell
  // The two volume parts, in the order that keeps the fewest values live:
  // FP64 the v-terms first (zv ends there), FP32 the x-terms first.
  auto vvolume = [&]() {
  // ---- volume, v-dimensions ----
  // B^-1(x3) [sum_j E_j(g) (Dt along v_j) Ux / h_j], Ux = B(x3) u: the
  // derivatives along v_j commute with the x-transform, which is applied once.
  {
    P ux[16];
    {
      const P r0 = tB[i3 * 4], r1 = tB[i3 * 4 + 1], r2 = tB[i3 * 4 + 2], r3 = tB[i3 * 4 + 3];
#pragma unroll
      for (int s = 0; s < 16; ++s)
        ux[s] = r0 * cellb[off3 + 256 * s] + r1 * cellb[off3 + 16 + 256 * s] +
                r2 * cellb[off3 + 32 + 256 * s] + r3 * cellb[off3 + 48 + 256 * s];
    }
    k3g_lane<1, 16>(tB, ux, l);
    k3g_lane<2, 16>(tB, ux, l);
    // Ux to LDS for the derivative across the waves (the face layers are
    // consumed: every wave passed the barrier below only after its reads)
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) faceb[t + 256 * s] = ux[s];
    __syncthreads();
    const P c4 = prm.inv_h[3] * eg[0], c5 = prm.inv_h[4] * eg[1], c6 = prm.inv_h[5] * eg[2];
    P z[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i5 = s & 3, i6 = s >> 2;
      P d4 = P(0), d5 = P(0), d6 = P(0);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) {
        d4 += tDt[w * 4 + mm] * faceb[l + 64 * mm + 256 * s];
        d5 += gt.Dt[i5 * 4 + mm] * ux[4 * i6 + mm];
        d6 += gt.Dt[i6 * 4 + mm] * ux[i5 + 4 * mm];
      }
      z[s] = c4 * d4 + c5 * d5 + c6 * d6;
      if constexpr (kMergeV) z[s] += zv[s];
    }
    k3g_lane<3, 16>(tBinv, z, l);
    k3g_lane<2, 16>(tBinv, z, l);
    k3g_lane<1, 16>(tBinv, z, l);
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[s] -= z[s];
  }

  };
  auto xvolume = [&]() {
  // ---- volume, x-dimensions: (alpha I + vh G) along v_j, Dt along x_j ----
  {
    // j = 0: G along i4 (waves, from LDS), Dt along i1
    P y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      P g4 = P(0);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) g4 += tG[w * 4 + mm] * cellb[l + 64 * mm + 256 * s];
      y[s] = alpha[0] * u[s] + vhh[0] * g4;
    }
    k3g_lane<1, 16>(tDt, y, l);
    const P ih = prm.inv_h[0];
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[s] -= ih * y[s];
  }
  {
    // j = 1: G along i5 (registers), Dt along i2
    P y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i5 = s & 3, s0 = s - i5;
      P g5 = P(0);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) g5 += gt.G[i5 * 4 + mm] * u[s0 + mm];
      y[s] = alpha[1] * u[s] + vhh[1] * g5;
    }
    k3g_lane<2, 16>(tDt, y, l);
    const P ih = prm.inv_h[1];
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[s] -= ih * y[s];
  }
  {
    // j = 2: Dt along i3 (lanes 16 apart, from LDS), then G along i6
    const P r0 = tDt[i3 * 4], r1 = tDt[i3 * 4 + 1], r2 = tDt[i3 * 4 + 2], r3 = tDt[i3 * 4 + 3];
    P y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
      y[s] = r0 * cellb[off3 + 256 * s] + r1 * cellb[off3 + 16 + 256 * s] +
             r2 * cellb[off3 + 32 + 256 * s] + r3 * cellb[off3 + 48 + 256 * s];
    const P ih = prm.inv_h[2];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i6 = s >> 2, s0 = s & 3;
      P g6 = P(0);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) g6 += gt.G[i6 * 4 + mm] * y[s0 + 4 * mm];
      acc[s] -= ih * (alpha[2] * y[s] + vhh[2] * g6);
    }
  }
  };
  if constexpr (kMergeV) {
    vvolume();
    xvolume();
  } else {
    xvolume();
    vvolume();
  }

  // ---- output / RK update ----
  const bool stage = prm.mode == 1;
  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
#pragma unroll
    for (int s = 0; s < 16; ++s) ocell[t + 256 * s] = acc[s];
    return;
  }
  P *ducell = prm.du + (uint64_t)cell * ND;
  P dv[16];
  if (prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.rk_a * ld_opt<NT>(ducell + t + 256 * s) + prm.dt * acc[s];
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.dt * acc[s];
  }
  if (prm.write_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) st_opt<NT>(ducell + t + 256 * s, dv[s]);
  }
  double *uocell = prm.u_out + (uint64_t)cell * ND;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    double uo;
    if constexpr (sizeof(P) == sizeof(double)) uo = (double)u[s];
    else uo = ucell[t + 256 * s];
    st_opt<NT>(uocell + t + 256 * s, uo + prm.rk_b * (double)dv[s]);
  }
}

}  // namespace hd
