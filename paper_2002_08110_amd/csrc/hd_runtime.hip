// C ABI of the library (declared in include/hd.h): solver objects, argument
// checking, workspace layout, field tables, initial states, the fused RK
// stage launches, hipGraph capture of whole RK steps, deterministic FP64
// diagnostics (batched stepping is in hd_batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "hd_internal.h"
#include "stage_gauss.h"
#include "stage_k3_gauss.h"
#include "stage_k3_mapped.h"
#include "stage_k3_mgauss.h"
#include "stage_dispatch.h"
#include "stage_k3.h"

namespace hd {
namespace rt {

thread_local std::string g_err;

hd_status fail(hd_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage scheme,
// the low-storage RK scheme of Sec. 5.4 (order 4, 5 stages, 3 vectors).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

}  // namespace rt
}  // namespace hd

namespace {

using hd::rt::fail;
using hd::rt::fill_params;
using hd::rt::k3_eligible;
using hd::rt::split_eligible;
using hd::rt::split_shapes;
using hd::rt::split_used;
using hd::rt::SplitShapes;
using hd::rt::kRkA;
using hd::rt::kRkB;

constexpr size_t kAlign = 256;
constexpr int kDiagBlocks = 1024;
constexpr int kDiagThreads = 256;
// Largest mesh of the allocation-free diagnostics: 2^40 DoFs, so that a block's
// chunk (ndofs / 1024) stays within 2^30 values.
constexpr long long kNoAllocMaxDofs = 1LL << 40;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace



namespace {

bool valid_plan(const hd_solver *s, const hd_plan &p, std::string *why) {
  if (p.options < 0 || p.options > 3) {
    *why = "options is a 2-bit mask";
    return false;
  }
  if (p.kernel < 0 || p.kernel > 2) {
    *why = "kernel must be 0 (generic), 1 (6D degree-3) or 2 (dimension-split)";
    return false;
  }
  if (p.kernel == 1) {
    if (!k3_eligible(s)) {
      *why = "kernel 1 needs d = 6 (3 x + 3 v) and degree 3";
      return false;
    }
    return true;
  }
  if (p.kernel == 2) {
    if (!split_eligible(s)) {
      *why = "kernel 2 needs d = 6 (3 x + 3 v) or d = 5 (3 x + 2 v) at degree 4 or 5, "
             "collocation on Cartesian cells";
      return false;
    }
    return true;
  }
  const int rd = p.reg_dims, sd = p.split_dims, ld = p.loop_dims;
  if (rd < 1 || rd > 2 || rd > s->dv) {
    *why = "reg_dims must be 1 or 2 and at most dim_v";
    return false;
  }
  if (sd < 0 || sd > 2 || (sd > 0 && (!p.lds || rd + sd > s->dv || s->n < 5 || s->d < 5))) {
    *why = "split_dims must be 0, 1 or 2, with lds = 1, reg_dims + split_dims <= dim_v, "
           "degree >= 4 and d >= 5";
    return false;
  }
  if (ld < 0 || ld > 1 || (ld == 1 && (!p.lds || p.cells_per_wg != 1))) {
    *why = "loop_dims must be 0 or 1; 1 needs lds = 1 and cells_per_wg = 1";
    return false;
  }
  int64_t T = 1, unit = 1;  // threads and nodes of one unit (cell or slab)
  for (int j = 0; j < s->d - rd - sd - ld; ++j) T *= s->n;
  for (int j = 0; j < s->d - sd; ++j) unit *= s->n;
  if (p.lds) {
    const int64_t unit_bytes = unit * (int64_t)s->psize();
    if (T > 1024 || p.cells_per_wg < 1 || p.cells_per_wg * T > 1024 ||
        p.cells_per_wg * unit_bytes > (int64_t)hd::kMaxLdsBytes) {
      *why = "LDS plan does not fit (threads <= 1024, LDS <= 160 KiB per workgroup)";
      return false;
    }
    if (T > 256 && p.cells_per_wg != 1) {
      *why = "units with more than 256 pencils take one unit per workgroup";
      return false;
    }
    if (T <= 256 && p.cells_per_wg * T > 256) {
      *why = "workgroups of units with <= 256 pencils hold at most 256 threads";
      return false;
    }
  } else {
    if (p.wg_size < 64 || p.wg_size > 256 || p.wg_size % 64) {
      *why = "wg_size must be 64, 128, 192 or 256";
      return false;
    }
  }
  // The variant must be compiled.
  hd_solver probe;
  probe.d = s->d;
  probe.dx = s->dx;
  probe.n = s->n;
  probe.prec = s->prec;
  probe.plan = p;
  if (!hd::rt::stage_entry(&probe)) {
    *why = "no compiled kernel variant for this plan";
    return false;
  }
  return true;
}

hd_plan default_plan(const hd_solver *s) {
  hd_plan p{};
  p.xcd_remap = 1;
  p.wg_size = 256;
  // Measured on MI355X: FP64 prefers two register dimensions up to degree 3
  // (16 nodes per thread), FP32 one.
  p.reg_dims = (s->dv >= 2 && (s->n <= 3 || (s->n == 4 && s->prec == HD_FP64))) ? 2 : 1;
  // Cells too large for LDS at degree 5 (d = 5, 6), and 6D degree 4 in
  // FP64: slabs along a velocity dimension and/or threads that loop over
  // the pencils of the first velocity dimension (measured on MI355X).
  if (s->n == 6 && s->d == 6) {
    p.reg_dims = 1;
    p.split_dims = 1;
    p.loop_dims = 1;
  } else if (s->n == 6 && s->d == 5) {
    p.reg_dims = 1;
    p.loop_dims = 1;
  } else if (s->n == 5 && s->d == 6 && s->prec == HD_FP64) {
    p.reg_dims = 2;
    p.split_dims = 1;
  } else if (s->n == 5 && s->d == 6) {
    p.reg_dims = 2;
  }
  int64_t T = 1, unit = 1;  // threads and nodes of one unit
  for (int j = 0; j < s->d - p.reg_dims - p.split_dims - p.loop_dims; ++j) T *= s->n;
  for (int j = 0; j < s->d - p.split_dims; ++j) unit *= s->n;
  const int64_t unit_bytes = unit * (int64_t)s->psize();
  if (T <= 1024 && unit_bytes <= (int64_t)hd::kMaxLdsBytes) {
    p.lds = 1;
    int cpw = (T <= 256 && !p.loop_dims) ? (int)(256 / T) : 1;
    while (cpw > 1 && cpw * unit_bytes > (int64_t)hd::kMaxLdsBytes) --cpw;
    p.cells_per_wg = std::max(1, cpw);
  } else {
    p.lds = 0;
    p.split_dims = 0;
    p.loop_dims = 0;
    p.cells_per_wg = 1;
  }
  p.kernel = k3_eligible(s) ? 1 : 0;
  // Measured on MI355X (6D 8^6, k = 3): streaming du and the output solution
  // helps both precisions, keeping the FP64 input in registers helps FP32.
  // The generic kernel streams them once the vectors outgrow the caches
  // (the autotuner picked streaming for most (d, k) at 1.5e8 DoFs).
  if (p.kernel == 1) p.options = s->prec == HD_FP32_OP_FP64_ACC ? 3 : 1;
  else p.options = s->ndofs >= (int64_t(1) << 25) ? 1 : 0;
  // Cell order of the 6D degree-3 kernel (measured on MI355X over 4^6 to
  // 9^6 and mixed meshes, with data of full entropy): in FP64 from about
  // 1e5 cells on, handing consecutive cells to the XCDs in turn keeps all of
  // them inside one window whose neighbour layers the shared last-level
  // cache still holds (8^6: 10% faster than contiguous slabs per XCD);
  // smaller meshes and the FP32 mode run faster with the slabs.
  if (p.kernel == 1 && s->prec == HD_FP64 && s->ncells >= 100000) p.xcd_remap = 0;
  return p;
}

}  // namespace

hd::LaunchShape hd::rt::shape_of(const hd_solver *s) {
  hd::LaunchShape ls{};
  if (hd::rt::k3g_used(s)) {
    ls.grid = (unsigned)s->ncells;
    ls.block = 256;
    ls.shmem = s->prec == HD_FP32_OP_FP64_ACC ? hd::k3g_lds_bytes<float>() : hd::k3g_lds_bytes<double>();
    return ls;
  }
  if (hd::rt::k3m_used(s)) {
    ls.grid = (unsigned)s->ncells;
    ls.block = 256;
    ls.shmem = s->prec == HD_FP32_OP_FP64_ACC ? hd::k3m_lds_bytes<float>() : hd::k3m_lds_bytes<double>();
    return ls;
  }
  if (hd::rt::k3mg_used(s)) {
    ls.grid = (unsigned)s->ncells;
    ls.block = 256;
    ls.shmem = s->prec == HD_FP32_OP_FP64_ACC ? hd::k3mg_lds_bytes<float>() : hd::k3mg_lds_bytes<double>();
    return ls;
  }
  if (s->quad == 1 || s->mapped()) {
    ls.grid = (unsigned)s->ncells;
    ls.block = (unsigned)hd::gauss_threads((int)s->nd);
    ls.shmem = (size_t)hd::gauss_lds_elems(s->d, s->n, s->dx, s->mapped(), (int)s->psize()) * s->psize();
    return ls;
  }
  if (s->plan.kernel == 1) {
    ls.grid = (unsigned)s->ncells;
    ls.block = 256;
    ls.shmem = s->prec == HD_FP32_OP_FP64_ACC ? hd::k3_lds_bytes<float>() : hd::k3_lds_bytes<double>();
    return ls;
  }
  if (s->plan.kernel == 2) return hd::rt::split_shapes(s).x;
  const int sd = s->plan.split_dims;
  int64_t T = 1, per_cell = 1;  // threads per unit, units per cell
  for (int j = 0; j < s->d - s->plan.reg_dims - sd - s->plan.loop_dims; ++j) T *= s->n;
  for (int j = 0; j < sd; ++j) per_cell *= s->n;
  if (s->plan.lds) {
    const int64_t cpw = s->plan.cells_per_wg;
    const int64_t units = s->ncells * per_cell;
    ls.grid = (unsigned)((units + cpw - 1) / cpw);
    ls.block = (unsigned)(cpw * T);
    ls.shmem = (size_t)(cpw * (s->nd / per_cell)) * s->psize();
  } else {
    const int64_t total = s->ncells * T;
    ls.grid = (unsigned)((total + s->plan.wg_size - 1) / s->plan.wg_size);
    ls.block = (unsigned)s->plan.wg_size;
    ls.shmem = 0;
  }
  return ls;
}

hd::rt::SplitShapes hd::rt::split_shapes(const hd_solver *s) {
  SplitShapes sh{};
  sh.e = hd::stage_split_entry(s->d, s->dx, s->n, s->prec == HD_FP32_OP_FP64_ACC, s->plan.options);
  if (!sh.e.fx) return sh;
  int64_t nvb = 1;
  for (int j = 0; j < s->dv; ++j) nvb *= s->n;
  const int64_t rows = s->ncells * nvb;
  sh.x.grid = (unsigned)((rows + sh.e.rows_per_tile - 1) / sh.e.rows_per_tile);
  sh.x.block = sh.e.threads_x;
  sh.x.shmem = sh.e.lds_x;
  sh.v.grid = (unsigned)(s->ncells * sh.e.tiles_per_cell);
  sh.v.block = sh.e.threads_v;
  sh.v.shmem = sh.e.lds_v;
  return sh;
}

namespace hd {
namespace rt {

const void *stage_entry(const hd_solver *s, int k3_role, int list) {
  const bool f32 = s->prec == HD_FP32_OP_FP64_ACC;
  if (list && !list_capable(s)) return nullptr;
  if (k3g_used(s)) return hd::stage_k3g_entry(f32);
  if (k3m_used(s)) return hd::stage_k3m_entry(f32);
  if (k3mg_used(s)) return hd::stage_k3mg_entry(f32);
  if (s->quad == 1 || s->mapped()) return hd::stage_gauss_entry(s->d, s->n, f32, s->mapped());
  if (s->plan.kernel == 1) return f32 ? hd::stage_k3_f32(s->plan.options, k3_role, list)
                                      : hd::stage_k3_f64(s->plan.options, k3_role, list);
  if (s->plan.kernel == 2) {
    if (list) return nullptr;
    return hd::stage_split_entry(s->d, s->dx, s->n, f32, s->plan.options).fx;
  }
  const int rd = s->plan.reg_dims, lds = s->plan.lds, n = s->n, sd = s->plan.split_dims,
            opt = s->plan.options, ld = s->plan.loop_dims;
  switch (s->d) {
    case 2: return f32 ? hd::stage_d2_f32(n, rd, lds, sd, opt, ld, list) : hd::stage_d2_f64(n, rd, lds, sd, opt, ld, list);
    case 3: return f32 ? hd::stage_d3_f32(n, rd, lds, sd, opt, ld, list) : hd::stage_d3_f64(n, rd, lds, sd, opt, ld, list);
    case 4: return f32 ? hd::stage_d4_f32(n, rd, lds, sd, opt, ld, list) : hd::stage_d4_f64(n, rd, lds, sd, opt, ld, list);
    case 5: return f32 ? hd::stage_d5_f32(n, rd, lds, sd, opt, ld, list) : hd::stage_d5_f64(n, rd, lds, sd, opt, ld, list);
    case 6: return f32 ? hd::stage_d6_f32(n, rd, lds, sd, opt, ld, list) : hd::stage_d6_f64(n, rd, lds, sd, opt, ld, list);
  }
  return nullptr;
}

}  // namespace rt
}  // namespace hd

namespace {

// Supported field/mesh combinations for the split x/v dimensions: the d = 2..6
// splits 1+1, 2+1, 2+2, 3+2, 3+3 are compiled.
bool split_compiled(int dx, int dv) {
  return (dx == 1 && dv == 1) || (dx == 2 && dv == 1) || (dx == 2 && dv == 2) ||
         (dx == 3 && dv == 2) || (dx == 3 && dv == 3);
}

}  // namespace

// Lets a kernel use up to 160 KiB of dynamic LDS, once per kernel entry.
hipError_t hd::rt::allow_large_lds(const void *fn) {
  static std::mutex mu;
  static std::unordered_set<const void *> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count(fn)) return hipSuccess;
  // The dynamic limit is what the workgroup maximum leaves beside the
  // kernel's static LDS (e.g. a workgroup reduction's).
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, fn);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(hd::kMaxLdsBytes - fa.sharedSizeBytes));
  if (e == hipSuccess) done.insert(fn);
  return e;
}

namespace {

using hd::rt::allow_large_lds;

// The nodal-space matrices of the Gauss-Legendre form at degree 3 (host,
// FP64): Dt = B^-1 Dg B, G = B^-1 diag(g) B, B^-1 lift_s.
template <typename P>
void k3g_tables(const hd::GaussTables1D &g, hd::K3GaussTables<P> *kt) {
  double Dt[16], G[16];
  for (int i = 0; i < 4; ++i)
    for (int m = 0; m < 4; ++m) {
      double dt = 0.0, gg = 0.0;
      for (int q = 0; q < 4; ++q) {
        double dgb = 0.0;
        for (int r = 0; r < 4; ++r) dgb += g.Dg[q * 4 + r] * g.B[r * 4 + m];
        dt += g.Binv[i * 4 + q] * dgb;
        gg += g.Binv[i * 4 + q] * g.g[q] * g.B[q * 4 + m];
      }
      Dt[i * 4 + m] = dt;
      G[i * 4 + m] = gg;
    }
  for (int q = 0; q < 16; ++q) {
    kt->B[q] = (P)g.B[q];
    kt->Binv[q] = (P)g.Binv[q];
    kt->Dt[q] = (P)Dt[q];
    kt->G[q] = (P)G[q];
  }
  for (int sd = 0; sd < 2; ++sd)
    for (int i = 0; i < 4; ++i) {
      double b = 0.0;
      for (int q = 0; q < 4; ++q) b += g.Binv[i * 4 + q] * g.lift[sd][q];
      kt->Blift[sd][i] = (P)b;
    }
  for (int q = 0; q < 4; ++q) kt->g[q] = (P)g.g[q];
}

// Tables of the mapped Gauss-Legendre kernel in the 6D degree-3 layout: the
// nodal-form matrices of the Cartesian one, and the Gauss-point weak
// derivative, traces and lifts.
template <typename P>
void k3mg_tables(const hd::GaussTables1D &g, hd::K3MGaussTables<P> *mt) {
  hd::K3GaussTables<P> kt;
  k3g_tables(g, &kt);
  for (int q = 0; q < 16; ++q) {
    mt->B[q] = kt.B[q];
    mt->Binv[q] = kt.Binv[q];
    mt->Dt[q] = kt.Dt[q];
    mt->G[q] = kt.G[q];
  }
  for (int q = 0; q < 4; ++q)
    for (int m = 0; m < 4; ++m) mt->Dw[q * 4 + m] = (P)(g.Dg[m * 4 + q] * g.om[m] / g.om[q]);
  for (int sd = 0; sd < 2; ++sd)
    for (int i = 0; i < 4; ++i) {
      mt->Blift[sd][i] = kt.Blift[sd][i];
      mt->ext[sd][i] = (P)g.ext[sd][i];
      mt->lift[sd][i] = (P)g.lift[sd][i];
    }
  for (int q = 0; q < 4; ++q) mt->g[q] = kt.g[q];
}

}  // namespace

namespace hd {
namespace rt {

// Kernel parameters, launch shape and k3 role of one operator application
// (mode 0: out = L(in)) or fused RK stage (mode 1: in -> u_out) of s, as
// launch_op issues it.
template <typename P>
void fill_stage(const hd_solver *s, const double *in, void *out, double *u_out, int mode, int stage,
                double dt, hd::StageParams<P> *prm_out, hd::LaunchShape *ls_out, int *k3_role_out) {
  hd::StageParams<P> &prm = *prm_out;
  // The sweep kernel (Gauss-Legendre quadrature or mapped cells) reads the
  // fields in their own form, not the specialised kernel's.
  const bool k3g = hd::rt::k3g_used(s), k3m = hd::rt::k3m_used(s), k3mg = hd::rt::k3mg_used(s);
  const bool sweep = (s->quad == 1 || s->mapped()) && !k3g && !k3m && !k3mg;
  fill_params<P>(s, &prm, sweep ? 0 : s->plan.kernel);
  const hd::LaunchShape ls = hd::rt::shape_of(s);
  *ls_out = ls;
  prm.nblocks = ls.grid;
  prm.u_in = in;
  prm.mode = mode;
  // The increment buffer is always a valid address (operator applications
  // neither read nor write it; the 6D degree-3 kernel forms its address).
  prm.du = reinterpret_cast<P *>(s->du());
  if (mode == 0) {
    prm.out = reinterpret_cast<P *>(out);
  } else {
    prm.u_out = u_out;
    prm.du = reinterpret_cast<P *>(s->du());
    prm.read_du = stage > 0;    // A_1 = 0: the first stage needs no du
    prm.write_du = stage < 4;   // du is dead after the last stage
    prm.rk_a = (P)kRkA[stage];
    prm.rk_b = kRkB[stage];
    prm.dt = (P)dt;
  }
  // Variants of the 6D degree-3 kernel: the first stage reads no increment;
  // the late-increment variant serves the last stage (FP64) or every later
  // stage (FP32), where it measured faster than holding the increment
  // through the sweeps.
  const bool f32 = s->prec == HD_FP32_OP_FP64_ACC;
  const int k3_role = mode != 1 ? 0 : (!prm.read_du ? 1 : (f32 || !prm.write_du ? 2 : 0));
  // The plan's cell order governs the general variant. The FP64 first-stage
  // and late-increment variants measured faster with one slab per XCD at 8^6
  // on data of full entropy (5.86 against 6.00 ms and 5.50 against 5.55 ms),
  // where the general variant is 3% faster with the window order.
  if (!k3g && !k3m && !k3mg && !sweep && s->plan.kernel == 1 && !f32 && k3_role != 0) prm.xcd_remap = 1;
  // The mapped-cell collocation kernel reads every x-face neighbour layer
  // of its boundary lanes, which the slab of its own XCD keeps in that L2:
  // 8.5 against 10.0 ms per FP64 stage at 8^6 with the window order.
  if (k3m) prm.xcd_remap = 1;
  *k3_role_out = k3_role;
}

template void fill_stage<float>(const hd_solver *, const double *, void *, double *, int, int,
                                double, hd::StageParams<float> *, hd::LaunchShape *, int *);
template void fill_stage<double>(const hd_solver *, const double *, void *, double *, int, int,
                                 double, hd::StageParams<double> *, hd::LaunchShape *, int *);

}  // namespace rt
}  // namespace hd

namespace {

template <typename P>
hd_status launch_op(hd_solver *s, const double *in, void *out, double *u_out, int mode,
                    int stage, double dt, hipStream_t st) {
  hd::StageParams<P> prm;
  hd::LaunchShape ls;
  int k3_role = 0;
  hd::rt::fill_stage<P>(s, in, out, u_out, mode, stage, dt, &prm, &ls, &k3_role);
  if (ls.grid == 0) return HD_OK;
  if ((uint64_t)ls.grid * ls.block >= (uint64_t(1) << 32))
    return fail(HD_ERR_UNSUPPORTED, "stage launch exceeds 2^32 work-items; use a plan with more "
                                    "nodes per thread");
  const bool k3g = hd::rt::k3g_used(s), k3m = hd::rt::k3m_used(s), k3mg = hd::rt::k3mg_used(s);
  const void *fn = hd::rt::stage_entry(s, k3_role);
  if (!fn) return fail(HD_ERR_HIP, "no compiled stage kernel for this plan");
  if (s->field_kind == 2) {
    // The Vlasov-Poisson field of this stage's input, into the E table. The
    // first stage of a step reads the state; later stages take the density
    // from the velocity moments the previous stage's kernel wrote with its
    // output (so a captured step does not depend on what preceded it).
    const bool moments = mode == 1 && stage > 0 && s->vp_mom_src == in;
    const hd_status vr = hd::rt::vp_enqueue(s, in, st, moments);
    if (vr != HD_OK) return vr;
    if (mode == 1 && s->quad == 0 && !s->mapped() && s->plan.kernel == 1 && s->vp_mom_bytes)
      prm.vp_mom = s->vp_mom();
  }
  if (ls.shmem > 65536) {
    hipError_t ae = allow_large_lds(fn);
    if (ae != hipSuccess)
      return fail(HD_ERR_HIP, std::string("raising the LDS limit: ") + hipGetErrorString(ae));
  }
  hd::GaussTables<P> gt;
  hd::K3GaussTables<P> kt;
  hd::K3MappedTables<P> km;
  hd::K3MGaussTables<P> kmg;
  void *args[] = {&prm, k3g ? (void *)&kt : (k3m ? (void *)&km : (k3mg ? (void *)&kmg : (void *)&gt))};
  if (k3g) k3g_tables(s->gtab, &kt);
  if (k3mg) {
    k3mg_tables(s->gtab, &kmg);
    prm.xmetric = s->xmetric();
  }
  if (k3m) {
    // Dw = W^-1 D^T W of the Gauss-Lobatto collocation
    for (int q = 0; q < 4; ++q)
      for (int m = 0; m < 4; ++m) km.Dw[q * 4 + m] = (P)(s->tab.D[m * 4 + q] * s->tab.w[m] / s->tab.w[q]);
    km.winv = (P)(1.0 / s->tab.w[0]);
    prm.xmetric = s->xmetric();
  }
  else if (s->quad == 1 || s->mapped()) {
    const hd::GaussTables1D &src = s->quad == 1 ? s->gtab : s->gltab;
    const int n = s->n;
    for (int q = 0; q < n * n; ++q) {
      gt.B[q] = (P)src.B[q];
      gt.Binv[q] = (P)src.Binv[q];
      gt.Dg[q] = (P)src.Dg[q];
    }
    for (int q = 0; q < n; ++q) {
      gt.g[q] = (P)src.g[q];
      gt.om[q] = (P)src.om[q];
      for (int sd = 0; sd < 2; ++sd) {
        gt.ext[sd][q] = (P)src.ext[sd][q];
        gt.lift[sd][q] = (P)src.lift[sd][q];
      }
    }
    if (s->mapped()) prm.xmetric = s->xmetric();
  }
  if (split_used(s)) {
    // Pass x, then pass v (stage_split.h), each with its own grid.
    const SplitShapes sh = split_shapes(s);
    if ((uint64_t)sh.v.grid * sh.v.block >= (uint64_t(1) << 32))
      return fail(HD_ERR_UNSUPPORTED, "stage launch exceeds 2^32 work-items");
    prm.nblocks = sh.x.grid;
    hipError_t e = hipLaunchKernel(sh.e.fx, dim3(sh.x.grid), dim3(sh.x.block), args, sh.x.shmem, st);
    if (e == hipSuccess) {
      prm.nblocks = sh.v.grid;
      e = hipLaunchKernel(sh.e.fv, dim3(sh.v.grid), dim3(sh.v.block), args, sh.v.shmem, st);
    }
    if (e != hipSuccess) return fail(HD_ERR_HIP, std::string("stage kernel launch: ") + hipGetErrorString(e));
    return HD_OK;
  }
  hipError_t e = hipLaunchKernel(fn, dim3(ls.grid), dim3(ls.block), args, ls.shmem, st);
  if (e != hipSuccess) return fail(HD_ERR_HIP, std::string("stage kernel launch: ") + hipGetErrorString(e));
  if (mode == 1) s->vp_mom_src = prm.vp_mom ? u_out : nullptr;
  return HD_OK;
}

hd_status enqueue_stage(hd_solver *s, int stage, double dt, hipStream_t st) {
  const double *in = s->u(s->cur);
  double *out = s->u(1 - s->cur);
  hd_status r = s->prec == HD_FP32_OP_FP64_ACC ? launch_op<float>(s, in, nullptr, out, 1, stage, dt, st)
                                   : launch_op<double>(s, in, nullptr, out, 1, stage, dt, st);
  if (r == HD_OK) s->cur = 1 - s->cur;
  return r;
}

void drop_graphs(hd_solver *s) {
  // A replay may still run on the caller's stream: wait for it first.
  if (s->gpending && s->gdone) hipEventSynchronize(s->gdone);
  s->gpending = false;
  for (int i = 0; i < 2; ++i)
    if (s->gexec[i]) {
      hipGraphExecDestroy(s->gexec[i]);
      s->gexec[i] = nullptr;
    }
  s->gvalid = false;
}

// The solver's plan, field or memory changed: captured steps are stale.
void changed(hd_solver *s) {
  drop_graphs(s);
  ++s->version;
  s->vp_mom_src = nullptr;
}

hd_status check_bound(const hd_solver *s) {
  if (!s) return fail(HD_ERR_INVALID, "solver is NULL");
  if (!s->bound()) return fail(HD_ERR_INVALID, "solver has no bound memory (call hd_bind)");
  return HD_OK;
}

// ---------------------------------------------------------------------------
// Initial state (nodal interpolation) and diagnostics kernels.
// ---------------------------------------------------------------------------

struct GeomArgs {
  int d, dx, n;
  unsigned cells[6];
  double lo[6], hi[6], h[6];
  double xi[8], w[8];
  long long nd, ndofs;
  double eps;  // x-space deformation
};

// The deformation of the configuration box: x_m = X_m + eps L_m prod_k
// sin(theta_k), theta_k = 2 pi (X_k - lo_k) / L_k (m, k < dx); Jx = dx/dX.
__host__ __device__ inline void map_box_point(int dx, const double *lo, const double *hi,
                                              double eps, const double *X, double *x,
                                              double Jx[3][3]) {
  const double two_pi = 6.283185307179586476925286766559;
  double sn[3], cs[3], prod = 1.0;
  for (int k = 0; k < dx; ++k) {
    const double th = two_pi * (X[k] - lo[k]) / (hi[k] - lo[k]);
    sn[k] = sin(th);
    cs[k] = cos(th);
    prod *= sn[k];
  }
  for (int m = 0; m < dx; ++m) {
    const double Lm = hi[m] - lo[m];
    x[m] = X[m] + eps * Lm * prod;
    for (int k = 0; k < dx; ++k) {
      double p = cs[k];
      for (int r = 0; r < dx; ++r)
        if (r != k) p *= sn[r];
      Jx[m][k] = (m == k ? 1.0 : 0.0) + eps * Lm * two_pi / (hi[k] - lo[k]) * p;
    }
  }
}

__host__ __device__ inline double det_small(int n, const double A[3][3]) {
  if (n == 1) return A[0][0];
  if (n == 2) return A[0][0] * A[1][1] - A[0][1] * A[1][0];
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

__global__ void init_kernel(GeomArgs g, int kind, double alpha, double *u) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.ndofs) return;
  long long cell = i / g.nd, node = i - cell * g.nd;
  double x[6];
  for (int j = 0; j < g.d; ++j) {
    const int c = (int)(cell % g.cells[j]);
    cell /= g.cells[j];
    const int q = (int)(node % g.n);
    node /= g.n;
    x[j] = g.lo[j] + (c + g.xi[q]) * g.h[j];
  }
  if (g.eps != 0.0) {
    double X[3] = {x[0], x[1], x[2]}, J[3][3];
    map_box_point(g.dx, g.lo, g.hi, g.eps, X, x, J);
  }
  const double two_pi = 6.283185307179586476925286766559;
  double v;
  if (kind == 0) {
    v = 1.0;
    for (int j = 0; j < g.d; ++j) v *= sin(two_pi * (x[j] - g.lo[j]) / (g.hi[j] - g.lo[j]));
  } else {
    double v2 = 0.0;
    for (int j = g.dx; j < g.d; ++j) v2 += x[j] * x[j];
    const int dv = g.d - g.dx;
    v = (1.0 + alpha * cos(two_pi * (x[0] - g.lo[0]) / (g.hi[0] - g.lo[0]))) *
        pow(two_pi, -0.5 * dv) * exp(-0.5 * v2);
  }
  u[i] = v;
}

// Pass 1: block b reduces the contiguous chunk [b*chunk, (b+1)*chunk) in a
// fixed order (strided per thread, then a fixed tree), so the result is
// bitwise reproducible.
__global__ void __launch_bounds__(kDiagThreads) diag_kernel1(GeomArgs g, const double *u, long long chunk, double *part) {
  __shared__ double sm[2][kDiagThreads];
  const long long b0 = (long long)blockIdx.x * chunk;
  const long long b1 = min(b0 + chunk, g.ndofs);
  double m = 0.0, e = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    long long node = i % g.nd, cell = i / g.nd;
    double W = 1.0, X[3];
    for (int j = 0; j < g.d; ++j) {
      const int q = (int)(node % g.n);
      W *= g.h[j] * g.w[q];
      if (j < 3) X[j] = g.lo[j] + ((double)(cell % g.cells[j]) + g.xi[q]) * g.h[j];
      node /= g.n;
      cell /= g.cells[j];
    }
    if (g.eps != 0.0) {  // times det(dx/dX) at the node
      double x[3], J[3][3];
      map_box_point(g.dx, g.lo, g.hi, g.eps, X, x, J);
      W *= det_small(g.dx, J);
    }
    const double v = u[i];
    m += W * v;
    e += W * v * v;
  }
  sm[0][threadIdx.x] = m;
  sm[1][threadIdx.x] = e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sm[0][0];
    part[2 * blockIdx.x + 1] = sm[1][0];
  }
}

__global__ void __launch_bounds__(kDiagThreads) diag_kernel2(const double *part, int nparts, double *res) {
  __shared__ double sm[2][kDiagThreads];
  double m = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    m += part[2 * i];
    e += part[2 * i + 1];
  }
  sm[0][threadIdx.x] = m;
  sm[1][threadIdx.x] = e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    res[0] = sm[0][0];
    res[1] = sm[1][0];
  }
}

GeomArgs geom_of(const hd_solver *s) {
  GeomArgs g{};
  g.d = s->d;
  g.dx = s->dx;
  g.n = s->n;
  for (int j = 0; j < s->d; ++j) {
    g.cells[j] = (unsigned)s->mesh.cells[j];
    g.lo[j] = s->mesh.lo[j];
    g.hi[j] = s->mesh.hi[j];
    g.h[j] = s->h[j];
  }
  for (int m = 0; m < s->n; ++m) {
    g.xi[m] = s->tab.xi[m];
    g.w[m] = s->tab.w[m];
  }
  g.nd = s->nd;
  g.ndofs = s->ndofs;
  g.eps = s->map_eps;
  return g;
}

// Metric of the mapped x-cells at the current quadrature points (layout of
// hd::gauss_metric_elems), uploaded to the device table.
hd_status upload_metric(hd_solver *s) {
  if (!s->mapped() || !s->bound()) return HD_OK;
  const int n = s->n, dx = s->dx;
  const double *pt = s->quad == 1 ? s->gtab.g : s->tab.xi;
  int64_t nxc = 1, nxn = 1;
  for (int j = 0; j < dx; ++j) {
    nxc *= s->mesh.cells[j];
    nxn *= n;
  }
  const int per = hd::gauss_metric_elems(n, dx), nfx = (int)(nxn / n);
  std::vector<double> tab((size_t)(nxc * per));
  // A = Jx diag(h_x) at the reference point xi of x-cell c: adj(A), det(A)
  auto metric = [&](const int *c, const double *xi, double adj[3][3], double *det) {
    double X[3] = {0, 0, 0}, x[3], J[3][3];
    for (int m = 0; m < dx; ++m) X[m] = s->mesh.lo[m] + (c[m] + xi[m]) * s->h[m];
    map_box_point(dx, s->mesh.lo, s->mesh.hi, s->map_eps, X, x, J);
    double A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int m = 0; m < dx; ++m)
      for (int k = 0; k < dx; ++k) A[m][k] = J[m][k] * s->h[k];
    *det = det_small(dx, A);
    if (dx == 1) {
      adj[0][0] = 1.0;
    } else if (dx == 2) {
      adj[0][0] = A[1][1];
      adj[0][1] = -A[0][1];
      adj[1][0] = -A[1][0];
      adj[1][1] = A[0][0];
    } else {
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
          const int r1 = (cc + 1) % 3, r2 = (cc + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
          adj[r][cc] = A[r1][c1] * A[r2][c2] - A[r1][c2] * A[r2][c1];
        }
    }
  };
  double dmin = 1e300;
  for (int64_t xc = 0; xc < nxc; ++xc) {
    int c[3] = {0, 0, 0};
    int64_t r = xc;
    for (int m = 0; m < dx; ++m) {
      c[m] = (int)(r % s->mesh.cells[m]);
      r /= s->mesh.cells[m];
    }
    double *out = tab.data() + xc * per;
    for (int64_t xq = 0; xq < nxn; ++xq) {
      double xi[3] = {0, 0, 0}, adj[3][3], det;
      int64_t rr = xq;
      for (int m = 0; m < dx; ++m) {
        xi[m] = pt[rr % n];
        rr /= n;
      }
      metric(c, xi, adj, &det);
      dmin = std::min(dmin, det);
      for (int a = 0; a < dx; ++a)
        for (int b = 0; b < dx; ++b) out[xq * (dx * dx + 1) + a * dx + b] = adj[a][b];
      out[xq * (dx * dx + 1) + dx * dx] = det;
    }
    double *face = out + nxn * (dx * dx + 1);
    for (int j = 0; j < dx; ++j)
      for (int sd = 0; sd < 2; ++sd)
        for (int xp = 0; xp < nfx; ++xp) {
          double xi[3] = {0, 0, 0}, adj[3][3], det;
          int rr = xp;
          for (int m = 0; m < dx; ++m) {
            if (m == j) continue;
            xi[m] = pt[rr % n];
            rr /= n;
          }
          xi[j] = sd ? 1.0 : 0.0;
          metric(c, xi, adj, &det);
          dmin = std::min(dmin, det);
          for (int k = 0; k < dx; ++k) face[((j * 2 + sd) * nfx + xp) * dx + k] = adj[j][k];
        }
  }
  if (!(dmin > 0.0)) return fail(HD_ERR_INVALID, "the mapping is not invertible on this mesh");
  HD_HIP(hipMemcpy(s->xmetric(), tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  return HD_OK;
}

// Device E table: the phase-space E at the x-nodes, or for a constant field
// the constant a_v at every x-node (read by the specialised kernel).
hd_status upload_E(hd_solver *s) {
  const size_t n = (size_t)s->nE;
  if (s->field_kind == 2) {
    // the table follows the state; only the transform matrices are uploaded
    const hd_status r = hd::rt::vp_upload(s);
    changed(s);
    return r;
  }
  if (s->field_kind == 0) {
    s->E_host.assign(n, 0.0);
    for (size_t i = 0; i < n; ++i) s->E_host[i] = s->a_const[s->dx + (int)(i % (size_t)s->dx)];
  }
  if (s->prec == HD_FP32_OP_FP64_ACC) {
    std::vector<float> tmp(s->E_host.begin(), s->E_host.end());
    HD_HIP(hipMemcpy(s->E(), tmp.data(), n * sizeof(float), hipMemcpyHostToDevice));
  } else {
    HD_HIP(hipMemcpy(s->E(), s->E_host.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }
  changed(s);
  return HD_OK;
}

// Plain streaming copy, 16 bytes per lane per iteration.
__global__ void __launch_bounds__(256) stream_copy_kernel(const double2 *__restrict__ src,
                                                          double2 *__restrict__ dst, size_t n2) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    dst[i] = src[i];
}

__global__ void stream_copy_tail(const double *src, double *dst, size_t begin, size_t n) {
  const size_t i = begin + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

// ===========================================================================
// ABI
// ===========================================================================

hd_status hd::rt::enqueue_stage_of(hd_solver *s, int par, int stage, double dt, hipStream_t st) {
  return s->prec == HD_FP32_OP_FP64_ACC
             ? launch_op<float>(s, s->u(par), nullptr, s->u(1 - par), 1, stage, dt, st)
             : launch_op<double>(s, s->u(par), nullptr, s->u(1 - par), 1, stage, dt, st);
}

hd_status hd::rt::enqueue_step(hd_solver *s, int par, double dt, hipStream_t st) {
  for (int stage = 0; stage < 5; ++stage, par = 1 - par) {
    const hd_status r =
        s->prec == HD_FP32_OP_FP64_ACC ? launch_op<float>(s, s->u(par), nullptr, s->u(1 - par), 1, stage, dt, st)
                           : launch_op<double>(s, s->u(par), nullptr, s->u(1 - par), 1, stage, dt, st);
    if (r != HD_OK) return r;
  }
  return HD_OK;
}

extern "C" {

const char *hd_last_error(void) { return hd::rt::g_err.c_str(); }

hd_status hd_create(const hd_mesh *mesh, int degree, int prec, hd_solver **out) {
  if (!mesh || !out) return fail(HD_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (mesh->dim_x < 1 || mesh->dim_x > 3 || mesh->dim_v < 1 || mesh->dim_v > 3)
    return fail(HD_ERR_INVALID, "dim_x and dim_v must be in 1..3");
  if (degree < 1) return fail(HD_ERR_INVALID, "degree must be >= 1");
  if (prec != HD_FP64 && prec != HD_FP32_OP_FP64_ACC) return fail(HD_ERR_INVALID, "unknown precision");
  const int d = mesh->dim_x + mesh->dim_v;
  long double cells_total = 1.0L;
  for (int j = 0; j < d; ++j) {
    if (mesh->cells[j] < 1) return fail(HD_ERR_INVALID, "cell counts must be >= 1");
    if (!(mesh->hi[j] > mesh->lo[j]) || !std::isfinite(mesh->lo[j]) || !std::isfinite(mesh->hi[j]))
      return fail(HD_ERR_INVALID, "need finite lo < hi in every dimension");
    cells_total *= mesh->cells[j];
  }
  if (degree > 5) return fail(HD_ERR_UNSUPPORTED, "degrees 1..5 are compiled");
  if (!split_compiled(mesh->dim_x, mesh->dim_v))
    return fail(HD_ERR_UNSUPPORTED,
                "compiled x+v splits are 1+1, 2+1, 2+2, 3+2, 3+3 (dim_x >= dim_v)");
  if (cells_total >= 4294967296.0L) return fail(HD_ERR_INVALID, "more than 2^32-1 cells");
  hd_solver *s = new (std::nothrow) hd_solver();
  if (!s) return fail(HD_ERR_OOM, "host allocation failed");
  s->mesh = *mesh;
  s->dx = mesh->dim_x;
  s->dv = mesh->dim_v;
  s->d = d;
  s->k = degree;
  s->n = degree + 1;
  s->prec = prec;
  s->nd = 1;
  s->ncells = 1;
  for (int j = 0; j < d; ++j) {
    s->nd *= s->n;
    s->ncells *= mesh->cells[j];
    s->h[j] = (mesh->hi[j] - mesh->lo[j]) / mesh->cells[j];
  }
  s->ndofs = s->nd * s->ncells;
  if (!hd::make_tables(degree, &s->tab)) {
    delete s;
    return fail(HD_ERR_INVALID, "Gauss-Lobatto table construction failed");
  }
  s->gtab_ok = hd::make_gauss_tables(s->tab, &s->gtab);
  hd::make_gl_quad_tables(s->tab, &s->gltab);
  int64_t nxc = 1, nxn = 1;
  for (int j = 0; j < s->dx; ++j) {
    nxc *= mesh->cells[j];
    nxn *= s->n;
  }
  s->nE = nxc * nxn * s->dx;
  const size_t N = (size_t)s->ndofs;
  size_t off = 0;
  s->off_u[0] = off;
  off = align_up(off + N * sizeof(double));
  s->off_u[1] = off;
  off = align_up(off + N * sizeof(double));
  s->state_total = off;
  off = 0;
  s->off_du = off;
  off = align_up(off + N * s->psize());
  s->off_E = off;
  off = align_up(off + (size_t)s->nE * s->psize());
  s->off_part = off;
  off = align_up(off + sizeof(double) * (2 * kDiagBlocks + 2));
  off = hd::rt::vp_layout(s, off);
  s->off_xmetric = off;
  off = align_up(off + sizeof(double) * (size_t)(nxc * hd::gauss_metric_elems(s->n, s->dx)));
  s->total = off;
  s->plan = default_plan(s);
  *out = s;
  return HD_OK;
}

hd_status hd_destroy(hd_solver *s) {
  if (!s) return HD_OK;
  drop_graphs(s);
  if (s->gdone) hipEventDestroy(s->gdone);
  if (s->cap) hipStreamDestroy(s->cap);
  delete s;
  return HD_OK;
}

hd_status hd_num_dofs(const hd_solver *s, int64_t *ndofs) {
  if (!s || !ndofs) return fail(HD_ERR_INVALID, "NULL argument");
  *ndofs = s->ndofs;
  return HD_OK;
}

hd_status hd_required_bytes(const hd_solver *s, size_t *state_bytes, size_t *workspace_bytes) {
  if (!s || !state_bytes || !workspace_bytes) return fail(HD_ERR_INVALID, "NULL argument");
  *state_bytes = s->state_total;
  *workspace_bytes = s->total;
  return HD_OK;
}

hd_status hd_bind(hd_solver *s, void *state_dev, size_t state_bytes, void *workspace_dev,
                  size_t workspace_bytes) {
  if (!s || !state_dev || !workspace_dev) return fail(HD_ERR_INVALID, "NULL argument");
  if (state_bytes < s->state_total)
    return fail(HD_ERR_INVALID, "state buffer smaller than hd_required_bytes");
  if (workspace_bytes < s->total)
    return fail(HD_ERR_INVALID, "workspace smaller than hd_required_bytes");
  if ((reinterpret_cast<uintptr_t>(state_dev) | reinterpret_cast<uintptr_t>(workspace_dev)) % kAlign)
    return fail(HD_ERR_INVALID, "state and workspace must be 256-byte aligned");
  const char *sb = reinterpret_cast<const char *>(state_dev);
  const char *wb = reinterpret_cast<const char *>(workspace_dev);
  if (sb < wb + s->total && wb < sb + s->state_total)
    return fail(HD_ERR_INVALID, "state and workspace must not overlap");
  changed(s);
  s->state = reinterpret_cast<char *>(state_dev);
  s->ws = reinterpret_cast<char *>(workspace_dev);
  s->cur = 0;
  HD_HIP(hipMemset(s->state, 0, s->state_total));
  HD_HIP(hipMemset(s->ws, 0, s->total));
  hd_status r = upload_metric(s);
  if (r) return r;
  return upload_E(s);
}

hd_status hd_set_field_constant(hd_solver *s, const double *a) {
  if (!s || !a) return fail(HD_ERR_INVALID, "NULL argument");
  for (int j = 0; j < s->d; ++j)
    if (!std::isfinite(a[j])) return fail(HD_ERR_INVALID, "field must be finite");
  s->field_kind = 0;
  s->sine = false;
  for (int j = 0; j < 6; ++j) s->a_const[j] = j < s->d ? a[j] : 0.0;
  changed(s);
  if (s->bound()) return upload_E(s);
  return HD_OK;
}

}  // extern "C"

namespace {

// The phase-space field with table E (nE values) and sign; the caller has
// checked the solver.
hd_status set_phase_table(hd_solver *s, const double *E_host, double sign) {
  for (int64_t i = 0; i < s->nE; ++i)
    if (!std::isfinite(E_host[i])) return fail(HD_ERR_INVALID, "E must be finite");
  s->E_host.assign(E_host, E_host + s->nE);
  s->field_kind = 1;
  s->esign = sign;
  return upload_E(s);
}

// E_j = amp sin(2 pi (x_j - lo_j) / L_j) at the (mapped) configuration nodes.
std::vector<double> sine_table(const hd_solver *s, double amp) {
  std::vector<double> E((size_t)s->nE);
  int64_t nxc = 1, nxn = 1;
  for (int j = 0; j < s->dx; ++j) {
    nxc *= s->mesh.cells[j];
    nxn *= s->n;
  }
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t xc = 0; xc < nxc; ++xc)
    for (int64_t xn = 0; xn < nxn; ++xn) {
      int64_t cr = xc, nr = xn;
      for (int j = 0; j < s->dx; ++j) {
        const int c = (int)(cr % s->mesh.cells[j]);
        const int q = (int)(nr % s->n);
        cr /= s->mesh.cells[j];
        nr /= s->n;
        double x = s->mesh.lo[j] + (c + s->tab.xi[q]) * s->h[j];
        if (s->mapped()) {
          double X[3] = {0, 0, 0}, xm[3], J[3][3];
          int64_t cr2 = xc, nr2 = xn;
          for (int m = 0; m < s->dx; ++m) {
            X[m] = s->mesh.lo[m] + ((double)(cr2 % s->mesh.cells[m]) + s->tab.xi[nr2 % s->n]) * s->h[m];
            cr2 /= s->mesh.cells[m];
            nr2 /= s->n;
          }
          map_box_point(s->dx, s->mesh.lo, s->mesh.hi, s->map_eps, X, xm, J);
          x = xm[j];
        }
        E[(size_t)((xc * nxn + xn) * s->dx + j)] =
            amp * std::sin(two_pi * (x - s->mesh.lo[j]) / (s->mesh.hi[j] - s->mesh.lo[j]));
      }
    }
  return E;
}

}  // namespace

extern "C" {

hd_status hd_set_field_phase_space(hd_solver *s, const double *E_host, double sign) {
  if (!s || !E_host) return fail(HD_ERR_INVALID, "NULL argument");
  if (s->dx != s->dv) return fail(HD_ERR_INVALID, "phase-space field needs dim_x == dim_v");
  hd_status r = check_bound(s);
  if (r) return r;
  s->sine = false;
  return set_phase_table(s, E_host, sign);
}

hd_status hd_set_field_sine(hd_solver *s, double amp, double sign) {
  if (!s) return fail(HD_ERR_INVALID, "NULL argument");
  if (s->dx != s->dv) return fail(HD_ERR_INVALID, "phase-space field needs dim_x == dim_v");
  hd_status r = check_bound(s);
  if (r) return r;
  if (!std::isfinite(amp) || !std::isfinite(sign)) return fail(HD_ERR_INVALID, "amp and sign must be finite");
  const std::vector<double> E = sine_table(s, amp);
  r = set_phase_table(s, E.data(), sign);
  if (r) return r;
  s->sine = true;
  s->sine_amp = amp;
  s->sine_sign = sign;
  return HD_OK;
}

hd_status hd_set_field_vlasov_poisson(hd_solver *s, int modes) {
  if (!s) return fail(HD_ERR_INVALID, "NULL argument");
  if (s->dx != s->dv) return fail(HD_ERR_INVALID, "Vlasov-Poisson field needs dim_x == dim_v");
  if (s->mapped()) return fail(HD_ERR_UNSUPPORTED, "the Vlasov-Poisson field needs Cartesian cells");
  hd_status r = check_bound(s);
  if (r) return r;
  if (modes < 1 || modes > hd::rt::kVpMaxModes)
    return fail(HD_ERR_INVALID, "modes must be 1.." + std::to_string(hd::rt::kVpMaxModes));
  s->field_kind = 2;
  s->sine = false;
  s->esign = -1.0;
  s->vp_modes = modes;
  return upload_E(s);
}

hd_status hd_set_quadrature(hd_solver *s, int quadrature) {
  if (!s) return fail(HD_ERR_INVALID, "NULL argument");
  if (quadrature != 0 && quadrature != 1)
    return fail(HD_ERR_INVALID, "quadrature must be 0 (Gauss-Lobatto) or 1 (Gauss-Legendre)");
  if (quadrature == 1) {
    if (!s->gtab_ok) return fail(HD_ERR_INVALID, "Gauss-Legendre table construction failed");
    if (!hd::stage_gauss_entry(s->d, s->n, s->prec == HD_FP32_OP_FP64_ACC))
      return fail(HD_ERR_UNSUPPORTED,
                  "the Gauss-Legendre kernel holds two cell-sized arrays and a face layer in "
                  "LDS: this "
                  "(d, degree, precision) exceeds 160 KiB");
  }
  s->quad = quadrature;
  changed(s);
  return upload_metric(s);
}

hd_status hd_set_mapping(hd_solver *s, double eps) {
  if (!s) return fail(HD_ERR_INVALID, "NULL argument");
  if (!(std::fabs(eps) <= 0.05)) return fail(HD_ERR_INVALID, "|eps| must be at most 0.05");
  if (eps != 0.0 && s->field_kind == 2)
    return fail(HD_ERR_UNSUPPORTED, "the Vlasov-Poisson field needs Cartesian cells");
  if (eps != 0.0 && !hd::stage_gauss_entry(s->d, s->n, s->prec == HD_FP32_OP_FP64_ACC, true))
    return fail(HD_ERR_UNSUPPORTED,
                "the mapped-cell kernel holds two cell-sized arrays and a face layer in LDS: "
                "this (d, degree, precision) exceeds 160 KiB or is not compiled");
  const double old = s->map_eps;
  s->map_eps = eps;
  changed(s);
  hd_status r = upload_metric(s);
  if (r) {
    s->map_eps = old;
    return r;
  }
  // The sine field lives at the node positions, which moved.
  if (s->sine && s->field_kind == 1 && s->bound()) {
    const std::vector<double> E = sine_table(s, s->sine_amp);
    r = set_phase_table(s, E.data(), s->sine_sign);
  }
  return r;
}

hd_status hd_compute_field(hd_solver *s, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (s->field_kind != 2) return HD_OK;
  return hd::rt::vp_enqueue(s, s->u(s->cur), (hipStream_t)stream);
}

hd_status hd_get_field(hd_solver *s, double *E_host, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!E_host) return fail(HD_ERR_INVALID, "NULL argument");
  if (s->dx != s->dv) return fail(HD_ERR_INVALID, "the field table needs dim_x == dim_v");
  const hipStream_t st = (hipStream_t)stream;
  if (s->field_kind == 2) {
    r = hd::rt::vp_enqueue(s, s->u(s->cur), st);
    if (r) return r;
  }
  const size_t n = (size_t)s->nE;
  if (s->prec == HD_FP32_OP_FP64_ACC) {
    std::vector<float> tmp(n);
    HD_HIP(hipMemcpyAsync(tmp.data(), s->E(), n * sizeof(float), hipMemcpyDeviceToHost, st));
    HD_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < n; ++i) E_host[i] = tmp[i];
  } else {
    HD_HIP(hipMemcpyAsync(E_host, s->E(), n * sizeof(double), hipMemcpyDeviceToHost, st));
    HD_HIP(hipStreamSynchronize(st));
  }
  return HD_OK;
}

hd_status hd_set_state(hd_solver *s, const double *u, int u_is_device, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!u) return fail(HD_ERR_INVALID, "NULL state");
  s->vp_mom_src = nullptr;
  HD_HIP(hipMemcpyAsync(s->u(s->cur), u, sizeof(double) * (size_t)s->ndofs,
                        u_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        (hipStream_t)stream));
  return HD_OK;
}

hd_status hd_init_state(hd_solver *s, int kind, const double *params, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (kind != 0 && kind != 1) return fail(HD_ERR_INVALID, "initial state kind must be 0 or 1");
  const double alpha = (kind == 1 && params) ? params[0] : 0.0;
  s->vp_mom_src = nullptr;
  const GeomArgs g = geom_of(s);
  const unsigned blocks = (unsigned)((s->ndofs + 255) / 256);
  hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, g, kind, alpha,
                     s->u(s->cur));
  HD_HIP(hipGetLastError());
  return HD_OK;
}

hd_status hd_state_ptr(const hd_solver *s, void **ptr) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!ptr) return fail(HD_ERR_INVALID, "NULL argument");
  *ptr = s->u(s->cur);
  return HD_OK;
}

hd_status hd_get_state(const hd_solver *s, double *u_host, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!u_host) return fail(HD_ERR_INVALID, "NULL argument");
  HD_HIP(hipMemcpyAsync(u_host, s->u(s->cur), sizeof(double) * (size_t)s->ndofs,
                        hipMemcpyDeviceToHost, (hipStream_t)stream));
  HD_HIP(hipStreamSynchronize((hipStream_t)stream));
  return HD_OK;
}

hd_status hd_apply(hd_solver *s, const double *in, void *out, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!in || !out) return fail(HD_ERR_INVALID, "NULL argument");
  const char *ib = reinterpret_cast<const char *>(in);
  const char *ob = reinterpret_cast<const char *>(out);
  const size_t ibytes = sizeof(double) * (size_t)s->ndofs, obytes = s->psize() * (size_t)s->ndofs;
  if (ib < ob + obytes && ob < ib + ibytes) return fail(HD_ERR_INVALID, "in and out must not overlap");
  return s->prec == HD_FP32_OP_FP64_ACC ? launch_op<float>(s, in, out, nullptr, 0, 0, 0.0, (hipStream_t)stream)
                            : launch_op<double>(s, in, out, nullptr, 0, 0, 0.0, (hipStream_t)stream);
}

hd_status hd_stable_dt(const hd_solver *s, double cfl, double *dt) {
  if (!s || !dt) return fail(HD_ERR_INVALID, "NULL argument");
  if (!(cfl > 0)) return fail(HD_ERR_INVALID, "cfl must be > 0");
  // The Vlasov-Poisson field of the current state, computed on the null
  // stream (ordered after the work of blocking streams).
  std::vector<double> Evp;
  if (s->field_kind == 2) {
    Evp.resize((size_t)s->nE);
    hd_status r = hd_get_field(const_cast<hd_solver *>(s), Evp.data(), nullptr);
    if (r) return r;
  }
  const std::vector<double> &Et = s->field_kind == 2 ? Evp : s->E_host;
  double sum = 0.0;
  for (int j = 0; j < s->d; ++j) {
    double amax = 0.0;
    if (s->field_kind == 0) {
      amax = std::fabs(s->a_const[j]);
    } else if (j < s->dx) {
      const int m = s->dx + j;
      for (int c = 0; c < s->mesh.cells[m]; ++c)
        for (int q = 0; q < s->n; ++q)
          amax = std::max(amax, std::fabs(s->mesh.lo[m] + (c + s->tab.xi[q]) * s->h[m]));
    } else {
      for (int64_t t = j - s->dx; t < s->nE; t += s->dx)
        amax = std::max(amax, std::fabs(s->esign * Et[(size_t)t]));
    }
    sum += amax / s->h[j];
  }
  if (!(sum > 0)) return fail(HD_ERR_INVALID, "field is zero: no CFL time step");
  *dt = cfl / ((2.0 * s->k + 1.0) * sum);
  return HD_OK;
}

hd_status hd_rk_stage(hd_solver *s, int stage, double dt, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (stage < 0 || stage > 4) return fail(HD_ERR_INVALID, "stage must be 0..4");
  if (!std::isfinite(dt)) return fail(HD_ERR_INVALID, "dt must be finite");
  return enqueue_stage(s, stage, dt, (hipStream_t)stream);
}

hd_status hd_rk_step(hd_solver *s, double dt, int nsteps, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (nsteps < 0 || !std::isfinite(dt)) return fail(HD_ERR_INVALID, "need nsteps >= 0, finite dt");
  if (nsteps == 0) return HD_OK;
  if (!s->gvalid || s->gdt != dt) {
    drop_graphs(s);
    if (!s->cap) HD_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    const int cur0 = s->cur;
    for (int par = 0; par < 2; ++par) {
      s->cur = par;
      hipGraph_t g = nullptr;
      HD_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
      hd_status er = HD_OK;
      for (int st = 0; st < 5 && er == HD_OK; ++st) er = enqueue_stage(s, st, dt, s->cap);
      hipError_t ee = hipStreamEndCapture(s->cap, &g);
      if (er != HD_OK) {
        if (g) hipGraphDestroy(g);
        s->cur = cur0;
        return er;
      }
      if (ee != hipSuccess) {
        s->cur = cur0;
        return fail(HD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ee));
      }
      hipError_t ei = hipGraphInstantiate(&s->gexec[par], g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ei != hipSuccess) {
        s->cur = cur0;
        drop_graphs(s);
        return fail(HD_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
      }
    }
    s->cur = cur0;
    s->gdt = dt;
    s->gvalid = true;
  }
  if (!s->gdone) HD_HIP(hipEventCreateWithFlags(&s->gdone, hipEventDisableTiming));
  for (int i = 0; i < nsteps; ++i) {
    HD_HIP(hipGraphLaunch(s->gexec[s->cur], (hipStream_t)stream));
    s->cur = 1 - s->cur;  // five stages: the solution ends in the other buffer
  }
  HD_HIP(hipEventRecord(s->gdone, (hipStream_t)stream));
  s->gpending = true;
  return HD_OK;
}

hd_status hd_diagnostics(const hd_solver *s, double *mass, double *energy, hd_stream stream) {
  hd_status r = check_bound(s);
  if (r) return r;
  if (!mass || !energy) return fail(HD_ERR_INVALID, "NULL argument");
  const GeomArgs g = geom_of(s);
  const long long chunk = (s->ndofs + kDiagBlocks - 1) / kDiagBlocks;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(diag_kernel1, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, g, s->u(s->cur), chunk,
                     s->part());
  HD_HIP(hipGetLastError());
  hipLaunchKernelGGL(diag_kernel2, dim3(1), dim3(kDiagThreads), 0, st, s->part(), kDiagBlocks,
                     s->part() + 2 * kDiagBlocks);
  HD_HIP(hipGetLastError());
  double res[2];
  HD_HIP(hipMemcpyAsync(res, s->part() + 2 * kDiagBlocks, sizeof(res), hipMemcpyDeviceToHost, st));
  HD_HIP(hipStreamSynchronize(st));
  *mass = res[0];
  *energy = res[1];
  return HD_OK;
}

}  // extern "C"

namespace {

// Partial sums of the allocation-free diagnostics (hd_diagnostics_noalloc):
// one (mass, energy) pair per block of the first reduction pass. Each GPU
// holds its own copy of this array until the process ends; host code uses
// the device address taken with hipGetSymbolAddress, never the name.
constexpr int kScratchPairs = kDiagBlocks;
static __device__ __align__(256) double scratch[2 * kScratchPairs];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the current device, taken once per
// device (with that device current) and kept.
hd_status scratch_ptr(double **out) {
  int dev = -1;
  HD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(HD_ERR_UNSUPPORTED, "device ordinal beyond the scratch table (64 devices)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HD_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return HD_OK;
}

}  // namespace

extern "C" {

hd_status hd_diagnostics_noalloc(const hd_solver *s, const double *u_dev, double *res_dev,
                                 hd_stream stream) {
  if (!s || !u_dev || !res_dev) return fail(HD_ERR_INVALID, "NULL argument");
  // The first pass writes one pair per block; the array holds kScratchPairs.
  static_assert(kDiagBlocks <= kScratchPairs, "scratch holds every partial pair");
  if (s->ndofs > kNoAllocMaxDofs)
    return fail(HD_ERR_INVALID, "hd_diagnostics_noalloc: more than 2^40 DoFs (the limit of its "
                                "fixed 1024-block reduction)");
  double *part = nullptr;
  hd_status r = scratch_ptr(&part);
  if (r) return r;
  const GeomArgs g = geom_of(s);
  const long long chunk = (s->ndofs + kDiagBlocks - 1) / kDiagBlocks;
  hipStream_t st = (hipStream_t)stream;
  // Every pair is written by its block (empty chunks write zeros), so
  // nothing needs clearing between calls.
  hipLaunchKernelGGL(diag_kernel1, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, g, u_dev, chunk,
                     part);
  HD_HIP(hipGetLastError());
  hipLaunchKernelGGL(diag_kernel2, dim3(1), dim3(kDiagThreads), 0, st, part, kDiagBlocks, res_dev);
  HD_HIP(hipGetLastError());
  return HD_OK;
}

hd_status hd_stream_copy(const double *src, double *dst, size_t n, hd_stream stream) {
  if ((!src || !dst) && n) return fail(HD_ERR_INVALID, "NULL argument");
  if (n == 0) return HD_OK;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return fail(HD_ERR_INVALID, "src and dst must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const size_t n2 = n / 2;
  if (n2) {
    const unsigned blocks = (unsigned)std::min<size_t>((n2 + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(src), reinterpret_cast<double2 *>(dst), n2);
    HD_HIP(hipGetLastError());
  }
  if (n % 2) {
    hipLaunchKernelGGL(stream_copy_tail, dim3(1), dim3(64), 0, st, src, dst, 2 * n2, n);
    HD_HIP(hipGetLastError());
  }
  return HD_OK;
}

hd_status hd_get_plan(const hd_solver *s, hd_plan *plan) {
  if (!s || !plan) return fail(HD_ERR_INVALID, "NULL argument");
  *plan = s->plan;
  return HD_OK;
}

hd_status hd_set_plan(hd_solver *s, const hd_plan *plan) {
  if (!s || !plan) return fail(HD_ERR_INVALID, "NULL argument");
  std::string why;
  if (!valid_plan(s, *plan, &why)) return fail(HD_ERR_INVALID, why);
  s->plan = *plan;
  changed(s);
  return HD_OK;
}

}  // extern "C"

// Batched stepping is implemented in hd_batch.hip.
