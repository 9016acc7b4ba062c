// Fused LSRK stage for six dimensions (3 x + 3 v) at degree 3 (4 nodes per
// dimension, 4096 nodes per cell): one cell per 256-thread workgroup.
//
// Thread t = lane + 64 * wave owns the 16 nodes
//   (i1, i2, i3) = lane bits (2 each),  i4 = wave,  (i5, i6) = register index s.
// Derivative sweeps: dims 5 and 6 act on the thread's registers; dims 1 and 2
// exchange values between lanes of a wave with DPP (quad broadcast, row
// rotation); dims 3 and 4 read the cell staged in LDS. All global loads of a
// cell - its own values and the six inflow face layers of its neighbours -
// are issued before the first use, so the cell pays one memory latency; the
// stage increment follows and overlaps the arithmetic. The face layers are
// spread evenly over the threads. Those of dims 5 and 6 land in the threads
// that use them; those of dims 1 to 4 pass to their users through LDS, and
// the face terms are taken before the sweeps so that the cell can then
// overwrite the layers: 32 KiB of LDS per workgroup in FP64, which lets
// three workgroups share a CU.
//
// The operator is the one of stage_kernel.h (strong form of the collocated
// weak form, upwind inflow jump, diagonal inverse mass folded in); the RK
// update is fused the same way.
#pragma once

#include "stage_kernel.h"

namespace hd {

constexpr int kK3Nodes = 4096;
constexpr int kK3Face = 1024;
// LDS: the four face layers of dims 1 to 4, then the cell in the same space.
template <typename P>
constexpr size_t k3_lds_bytes() {
  return (size_t)kK3Nodes * sizeof(P);
}
static_assert(4 * kK3Face == kK3Nodes, "face layers and cell share the LDS");

// Cross-lane moves with every row and bank enabled: each lane reads a
// valid source lane under the patterns used here (quad permutations, row
// rotations), so no lane keeps a previous value and none is supplied (which
// spares a register initialisation per move and lets FP32 arithmetic take
// the pattern as an operand modifier).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, false));
}
// quad_perm [m, m, m, m]: every lane reads lane m of its group of four.
constexpr int quad_bcast(int m) { return m | (m << 2) | (m << 4) | (m << 6); }
// row_ror:n - lane p of a 16-lane row reads lane (p - n) mod 16.
constexpr int row_ror(int n) { return 0x120 + n; }

// Insert a zero base-4 digit at position j into the 5-digit face index p.
__device__ __forceinline__ int k3_face_node0(int p, int j) {
  const int lowmask = (1 << (2 * j)) - 1;
  return (p & lowmask) | ((p & ~lowmask) << 2);
}

// Stage roles, each compiled separately: the general kernel (operator
// application and stages; the increment loads overlap the sweeps), the
// first stage (no increment to read: its registers are free) and the
// late-increment kernel (the increment is loaded only for the update, which
// frees its registers during the sweeps; any stage after the first).
constexpr int kK3General = 0, kK3First = 1, kK3Last = 2;

// Register budget per thread. The general FP64 kernel holds the increment
// through the sweeps and runs 3 workgroups per CU = 3 waves per SIMD (at most
// 168 VGPRs; 4 would spill); without that, the first-stage and
// late-increment variants fit 128 VGPRs and run 4. FP32: 4 (5 would spill).
template <typename P, int ROLE>
constexpr int k3_waves_per_eu() {
  return sizeof(P) == 8 ? (ROLE == kK3General ? 3 : 4) : 4;
}

// Plan options (hd_plan.options): bit 0 (kOptStream, stage_kernel.h)
// streams du and the output solution with non-temporal accesses; bit 1
// (FP32) keeps the FP64 input solution in registers for the update instead
// of re-reading it.
constexpr int kOptKeepU64 = 2;

// One workgroup's cell `cell` (lds_reuse as in stage_body) in stage role
// ROLE; the first-stage role requires read_du == 0.
template <typename P, int OPT, int ROLE, typename PV = const StageParams<P>>
__device__ __forceinline__ void stage_k3_body(PV &prm, unsigned cell, unsigned char *smem_raw,
                                              bool lds_reuse, const int t) {
  constexpr bool NT = (OPT & kOptStream) != 0;
  constexpr bool KEEPU = (OPT & kOptKeepU64) != 0 && sizeof(P) == 4;
  constexpr bool EARLY_DU = ROLE == kK3General;  // increment loaded before the sweeps
  constexpr bool ANY_DU = ROLE != kK3First;
  constexpr int N = 4, ND = kK3Nodes, F = kK3Face;
  P *cellb = reinterpret_cast<P *>(smem_raw);
  P *faceb = cellb;  // layers of dims 1-4 first, then the cell
  const int l = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int i1 = l & 3, i2 = (l >> 2) & 3, i3 = l >> 4;

  unsigned c[6], left[6], right[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    c[j] = (cell / prm.cstride[j]) % prm.cells[j];
    const unsigned nj = prm.cells[j], st = prm.cstride[j];
    left[j] = c[j] == 0 ? cell + (nj - 1) * st : cell - st;
    right[j] = c[j] == nj - 1 ? cell - (nj - 1) * st : cell + st;
  }
  // Field: a_{x_j} = vlo + (c + xi) vh of velocity dim 3 + j, a_{v_j} =
  // esign * E_j at the x-node, which for this thread is its lane (i1,i2,i3).
  // A constant field is passed in the same form (vh = 0, E filled with the
  // constant), so the kernel has no field branch.
  const unsigned xcell = c[0] + prm.cells[0] * (c[1] + prm.cells[1] * c[2]);
  const P *e = prm.E + ((uint64_t)xcell * 64 + l) * 3;
  P ev[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) ev[j] = prm.esign * e[j];
  // a_{x_j} at velocity digit d: vb[j] + xi_d vh[j]. The one digit that
  // varies per lane in phase A uses a value loaded per lane once here (no
  // select chains, which the compiler turns into a lookup table in scratch).
  P vb[3], vhh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    vhh[j] = prm.vh[3 + j];
    vb[j] = prm.vlo[3 + j] + P(c[3 + j]) * vhh[j];
  }
  const P xi_i3 = prm.xi[i3];  // per lane
  auto ax = [&](int j, int digit) -> P { return vb[j] + prm.xi[digit] * vhh[j]; };

  // ---- phase A: issue every global load of the cell ----
  // Uniform (scalar) base pointers and 32-bit per-lane offsets keep the
  // address arithmetic out of the vector registers.
  const double *ucell = prm.u_in + (uint64_t)cell * ND;
  // Raw FP64 values; conversion to P waits until every load is issued.
  double ud[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) ud[s] = ucell[t + 256 * s];
  const bool stage = prm.mode == 1;
  // Neighbour cell offsets relative to this cell, in DoFs (uniform; the
  // library limits the state to fewer than 2^31 DoFs).
  int lofs[6], rofs[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    lofs[j] = ((int)left[j] - (int)cell) * ND;
    rofs[j] = ((int)right[j] - (int)cell) * ND;
  }
  // Inflow layers: face node p = t + 256 q of dimension j takes the left
  // neighbour's i_j = 3 value where a_j > 0 and the right neighbour's
  // i_j = 0 value where a_j < 0. The address is selected and the load always
  // issued (the own node where a_j = 0; its consumer weight is zero).
  double fv[6][4];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = t + 256 * q;
      const int node0 = k3_face_node0(p, j);
      // a_j at the face node: dim 1 at velocity digit i4 = digit 2 of p =
      // (t >> 4) & 3 (this lane's i3), dim 2 at i5 = digit 3 of p = wave,
      // dim 3 at i6 = digit 4 of p = q; the v dims at the x-node of the
      // face node, which is this lane's.
      P a;
      if (j == 0) a = vb[0] + xi_i3 * vhh[0];
      else if (j == 1) a = ax(1, w);
      else if (j == 2) a = ax(2, q);
      else a = ev[j - 3];
      const bool useL = a > P(0), useR = a < P(0);
      const int off = useL ? lofs[j] + node0 + 3 * (1 << (2 * j)) : (useR ? rofs[j] + node0 : node0);
      fv[j][q] = ucell[(long long)off];
    }
  }
  sched_fence();
  // ---- phase B: the face layers of dims 1-4 in LDS ----
  if (lds_reuse) __syncthreads();
  P u[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) u[s] = to_p<P>(ud[s]);
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) faceb[j * F + t + 256 * q] = to_p<P>(fv[j][q]);
  __syncthreads();
  // The stage increment is loaded now; its latency overlaps the arithmetic.
  P *ducell = prm.du + (uint64_t)cell * ND;
  P dv[16];
  if (EARLY_DU && stage && prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = ld_opt<NT>(ducell + t + 256 * s);
  }
  P acc[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) acc[s] = P(0);
#define Dm prm.Dm
  // ---- inflow faces ----
  // Branch-free: every thread reads the layer entry of each of its nodes and
  // weights it by zero unless the node lies on that dimension's inflow face.
  // Dims 1-4 read the layers from LDS, dims 5 and 6 from the registers that
  // loaded them: face node t + 256 q of dim 5 lies on this thread's nodes
  // s = 4 q (i5 = 0) and 4 q + 3 (i5 = 3), of dim 6 on s = q and 12 + q.
  {
    // dim 1: a = v_1(i4); face index p = node >> 2
    const P a = ax(0, w);
    const P wt = ((i1 == 0 && a > P(0)) ? a : ((i1 == 3 && a < P(0)) ? -a : P(0))) *
                 prm.lift_inv_h[0];
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[s] += wt * (faceb[0 * F + (t >> 2) + 64 * s] - u[s]);
  }
#pragma unroll
  for (int z = 0; z < 16; ++z) pin(acc[z]);
  sched_fence();
  {
    // dim 2: a = v_2(i5); p = (node & 3) + 4 (node >> 4)
    const int pb = (t & 3) + 4 * (t >> 4);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const P a = ax(1, s & 3);
      const P wt = ((i2 == 0 && a > P(0)) ? a : ((i2 == 3 && a < P(0)) ? -a : P(0))) *
                   prm.lift_inv_h[1];
      acc[s] += wt * (faceb[1 * F + pb + 64 * s] - u[s]);
    }
  }
#pragma unroll
  for (int z = 0; z < 16; ++z) pin(acc[z]);
  sched_fence();
  {
    // dim 3: a = v_3(i6); p = (node & 15) + 16 (node >> 6)
    const int pb = (t & 15) + 16 * (t >> 6);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const P a = ax(2, s >> 2);
      const P wt = ((i3 == 0 && a > P(0)) ? a : ((i3 == 3 && a < P(0)) ? -a : P(0))) *
                   prm.lift_inv_h[2];
      acc[s] += wt * (faceb[2 * F + pb + 64 * s] - u[s]);
    }
  }
#pragma unroll
  for (int z = 0; z < 16; ++z) pin(acc[z]);
  sched_fence();
  {
    // dim 4: a = E_1 (per lane), i4 = wave (uniform); p = l + 64 s
    const P a = ev[0];
    if (w == 0 || w == 3) {
      const P wt = ((w == 0 && a > P(0)) ? a : ((w == 3 && a < P(0)) ? -a : P(0))) *
                   prm.lift_inv_h[3];
#pragma unroll
      for (int s = 0; s < 16; ++s) acc[s] += wt * (faceb[3 * F + l + 64 * s] - u[s]);
    }
  }
#pragma unroll
  for (int z = 0; z < 16; ++z) pin(acc[z]);
  sched_fence();
  {
    // dim 5: i5 = s & 3, a = E_2; p = t + 256 i6; inflow node i5 = 0 (a > 0) or 3 (a < 0)
    const P a = ev[1];
    const P wl = a > P(0) ? a * prm.lift_inv_h[4] : P(0);
    const P wr = a < P(0) ? -a * prm.lift_inv_h[4] : P(0);
#pragma unroll
    for (int i6 = 0; i6 < 4; ++i6) {
      const P fvv = to_p<P>(fv[4][i6]);
      acc[4 * i6] += wl * (fvv - u[4 * i6]);
      acc[4 * i6 + 3] += wr * (fvv - u[4 * i6 + 3]);
    }
  }
  {
    // dim 6: i6 = s >> 2, a = E_3; p = t + 256 i5
    const P a = ev[2];
    const P wl = a > P(0) ? a * prm.lift_inv_h[5] : P(0);
    const P wr = a < P(0) ? -a * prm.lift_inv_h[5] : P(0);
#pragma unroll
    for (int i5 = 0; i5 < 4; ++i5) {
      const P fvv = to_p<P>(fv[5][i5]);
      acc[i5] += wl * (fvv - u[i5]);
      acc[12 + i5] += wr * (fvv - u[12 + i5]);
    }
  }

  // ---- the cell in LDS, over the consumed layers ----
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 16; ++s) cellb[t + 256 * s] = u[s];
  __syncthreads();
  // ---- phase C: sweeps ----
  // dims 5 and 6 (registers): a_{v_2} = ev[1], a_{v_3} = ev[2] are per thread
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int sstride = r == 0 ? 1 : 4;
    const P coef = -ev[1 + r] * prm.inv_h[4 + r];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int ij = (s / sstride) & 3;
      const int s0 = s - ij * sstride;
      P sum = Dm[ij * N] * u[s0];
#pragma unroll
      for (int m = 1; m < N; ++m) sum += Dm[ij * N + m] * u[s0 + m * sstride];
      acc[s] += coef * sum;
    }
  }
#pragma unroll
  for (int z = 0; z < 16; ++z) pin(acc[z]);
  sched_fence();
  // dim 1: lanes of a quad hold the line; a_{x_1} = v_1 at i4 = wave
  {
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = Dm[i1 * N + m];
    const P coef = -ax(0, w) * prm.inv_h[0];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      P sum = row[0] * dpp_move<quad_bcast(0)>(u[s]);
      sum += row[1] * dpp_move<quad_bcast(1)>(u[s]);
      sum += row[2] * dpp_move<quad_bcast(2)>(u[s]);
      sum += row[3] * dpp_move<quad_bcast(3)>(u[s]);
      acc[s] += coef * sum;
      if ((s & 3) == 3) {
#pragma unroll
        for (int z = s - 3; z <= s; ++z) pin(acc[z]);
        sched_fence();
      }
    }
  }
  sched_fence();
  // dim 2: lanes 4 apart in a row; rotation by 4n brings i2 - n
  {
    P rr[N];
#pragma unroll
    for (int n = 0; n < N; ++n) rr[n] = Dm[i2 * N + ((i2 - n) & 3)];
    const P ih = prm.inv_h[1];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      P sum = rr[0] * u[s];
      sum += rr[1] * dpp_move<row_ror(4)>(u[s]);
      sum += rr[2] * dpp_move<row_ror(8)>(u[s]);
      sum += rr[3] * dpp_move<row_ror(12)>(u[s]);
      acc[s] -= ax(1, s & 3) * ih * sum;
      if ((s & 3) == 3) {
#pragma unroll
        for (int z = s - 3; z <= s; ++z) pin(acc[z]);
        sched_fence();
      }
    }
  }
  sched_fence();
  // dim 3: LDS, lanes 16 apart
  {
    P row[N];
#pragma unroll
    for (int m = 0; m < N; ++m) row[m] = Dm[i3 * N + m];
    const P ih = prm.inv_h[2];
    const int off = (l & 15) + 64 * w;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      P sum = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) sum += row[m] * cellb[off + 16 * m + 256 * s];
      acc[s] -= ax(2, s >> 2) * ih * sum;
      if ((s & 3) == 3) {
#pragma unroll
        for (int z = s - 3; z <= s; ++z) pin(acc[z]);
        sched_fence();
      }
    }
  }
  sched_fence();
  // dim 4: LDS, across the four waves; a_{v_1} = ev[0]
  {
    const P coef = -ev[0] * prm.inv_h[3];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      P sum = P(0);
#pragma unroll
      for (int m = 0; m < N; ++m) sum += Dm[w * N + m] * cellb[l + 64 * m + 256 * s];
      acc[s] += coef * sum;
      if ((s & 3) == 3) {
#pragma unroll
        for (int z = s - 3; z <= s; ++z) pin(acc[z]);
        sched_fence();
      }
    }
  }
  sched_fence();
  // ---- phase D: output / RK update ----
  if (!stage) {
    P *ocell = prm.out + (uint64_t)cell * ND;
#pragma unroll
    for (int s = 0; s < 16; ++s) ocell[t + 256 * s] = acc[s];
    return;
  }
  if (!EARLY_DU && ANY_DU && prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = ld_opt<NT>(ducell + t + 256 * s);
  }
  if (ANY_DU && prm.read_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = rk_fma(prm.rk_a, dv[s], prm.dt * acc[s]);
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) dv[s] = prm.dt * acc[s];
  }
  if (prm.write_du) {
#pragma unroll
    for (int s = 0; s < 16; ++s) st_opt<NT>(ducell + t + 256 * s, dv[s]);
  }
  double *uocell = prm.u_out + (uint64_t)cell * ND;
  double mom = 0.0, mrow = 0.0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    double uo;
    if constexpr (sizeof(P) == sizeof(double)) uo = (double)u[s];
    else if constexpr (KEEPU) uo = ud[s];
    else uo = ucell[t + 256 * s];
    const double un = rk_fma(prm.rk_b, (double)dv[s], uo);
    st_opt<NT>(uocell + t + 256 * s, un);
    mrow += prm.gw[s & 3] * un;
    if ((s & 3) == 3) {
      mom += prm.gw[s >> 2] * mrow;
      mrow = 0.0;
    }
  }
  if (prm.vp_mom) prm.vp_mom[(uint64_t)cell * 256 + t] = mom;
}

template <typename P, int OPT, int ROLE>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(k3_waves_per_eu<P, ROLE>(), k3_waves_per_eu<P, ROLE>())))
    stage_k3_kernel(const StageParams<P> prm) {
  extern __shared__ unsigned char smem_raw[];
  unsigned cell = blockIdx.x;
  if (prm.xcd_remap) cell = xcd_tile(cell, prm.nblocks);
  stage_k3_body<P, OPT, ROLE>(prm, cell, smem_raw, false, (int)threadIdx.x);
}

// Work-list form (as stage_list_kernel): workgroup `item` runs the cell of
// the item's solve with that solve's parameters.
template <typename P, int OPT, int ROLE>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(k3_waves_per_eu<P, ROLE>(), k3_waves_per_eu<P, ROLE>())))
    stage_k3_list_kernel(const ListParams<P> lp) {
  extern __shared__ unsigned char smem_raw[];
  const unsigned item = blockIdx.x;
  const int slot = __builtin_amdgcn_readfirstlane(work_list_slot(lp.item0, lp.nslots, item));
  const unsigned t0 = __builtin_amdgcn_readfirstlane(item - lp.item0[slot]);
  ConstStageParams<P> &prm = lp.prm[slot];
  if (t0 >= prm.nblocks) return;  // padding: the whole workgroup
  const unsigned cell = prm.xcd_remap ? xcd_tile(t0, prm.nblocks) : t0;
  stage_k3_body<P, OPT, ROLE, ConstStageParams<P>>(prm, cell, smem_raw, false, (int)threadIdx.x);
}

#undef Dm
}  // namespace hd
