// Internal declarations shared by the library's translation units: the
// solver object, error reporting, RK coefficients and the kernel-parameter
// fill used by the single-solve and the batched launch paths.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "gl_tables.h"
#include "hd.h"
#include "stage_dispatch.h"
#include "stage_kernel.h"

struct hd_solver {
  hd_mesh mesh{};
  int d = 0, dx = 0, dv = 0, k = 0, n = 0, prec = 0;
  int64_t nd = 0, ncells = 0, ndofs = 0;
  double h[6] = {0};
  hd::Tables1D tab;
  int field_kind = 0;
  double a_const[6] = {0};
  double esign = 1.0;
  std::vector<double> E_host;  // E at x-nodes (phase-space field)
  int64_t nE = 0;              // entries of the E table
  // The prescribed sine field (hd_set_field_sine): its amplitude and sign,
  // kept so that a later mapping recomputes the table at the mapped nodes.
  bool sine = false;
  double sine_amp = 0.0, sine_sign = 1.0;
  // Caller-owned device memory: the state buffer holds the two FP64
  // solution vectors (offsets off_u), the workspace everything else
  // (offsets below), each section 256-byte aligned.
  size_t off_u[2] = {0, 0}, state_total = 0;
  size_t off_du = 0, off_E = 0, off_part = 0, total = 0;
  char *state = nullptr;
  char *ws = nullptr;
  bool bound() const { return state != nullptr && ws != nullptr; }
  int cur = 0;  // which of the two solution buffers holds the solution
  hd_plan plan{};
  // Captured RK steps (index = solution buffer parity at the start).
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  double gdt = 0.0;
  bool gvalid = false;
  // Recorded after the last replay of a captured step: a graph is destroyed
  // only once its launches have finished.
  hipEvent_t gdone = nullptr;
  bool gpending = false;
  uint64_t version = 0;  // bumped when the plan, field or memory changes
  // Quadrature: 0 Gauss-Lobatto collocation, 1 Gauss-Legendre (k+1 points).
  int quad = 0;
  hd::GaussTables1D gtab{};
  bool gtab_ok = false;
  hd::GaussTables1D gltab{};  // the collocation rule in the same form
  // Mapped configuration cells: deformation amplitude (0: Cartesian) and the
  // device metric table (hd::gauss_metric_elems per x-cell).
  double map_eps = 0.0;
  size_t off_xmetric = 0;
  bool mapped() const { return map_eps != 0.0; }
  // Vlasov-Poisson field (field_kind 2): modes per dimension and scratch.
  int vp_modes = 0, vp_groups = 0;
  size_t off_vp_partial = 0, off_vp_wv = 0, off_vp_A = 0, off_vp_B = 0, off_vp_Eh = 0,
         off_vp_mats = 0, off_vp_mom = 0;
  // Velocity moments written by the 6D degree-3 stage kernel (vp_mom_bytes
  // > 0 for such solvers) and the solution buffer they describe (null: none).
  size_t vp_mom_bytes = 0;
  const double *vp_mom_src = nullptr;

  double *u(int i) const { return reinterpret_cast<double *>(state + off_u[i]); }
  void *du() const { return ws + off_du; }
  void *E() const { return ws + off_E; }
  double *part() const { return reinterpret_cast<double *>(ws + off_part); }
  double *vp_partial() const { return reinterpret_cast<double *>(ws + off_vp_partial); }
  double *vp_wv() const { return reinterpret_cast<double *>(ws + off_vp_wv); }
  double2 *vp_bufA() const { return reinterpret_cast<double2 *>(ws + off_vp_A); }
  double2 *vp_bufB() const { return reinterpret_cast<double2 *>(ws + off_vp_B); }
  double2 *vp_Ehat() const { return reinterpret_cast<double2 *>(ws + off_vp_Eh); }
  double2 *vp_mats() const { return reinterpret_cast<double2 *>(ws + off_vp_mats); }
  double *vp_mom() const { return reinterpret_cast<double *>(ws + off_vp_mom); }
  double *xmetric() const { return reinterpret_cast<double *>(ws + off_xmetric); }
  size_t psize() const { return prec == HD_FP32_OP_FP64_ACC ? sizeof(float) : sizeof(double); }
};

#define HD_HIP(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return hd::rt::fail(HD_ERR_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

namespace hd {
namespace rt {

extern thread_local std::string g_err;
hd_status fail(hd_status st, const std::string &msg);
extern const double kRkA[5];
extern const double kRkB[5];

// The specialised kernel covers d = 6 (3 x + 3 v) at degree 3.
// Its in-kernel neighbour offsets are 32-bit DoF counts: fewer than 2^31 DoFs.
inline bool k3_eligible(const hd_solver *s) {
  return s->d == 6 && s->dx == 3 && s->n == 4 && s->ndofs < (int64_t(1) << 31);
}

// Gauss-Legendre quadrature on Cartesian cells runs in the 6D degree-3
// layout when the plan selects that kernel (kernel 0: the sweep kernel).
inline bool k3g_used(const hd_solver *s) {
  return s->quad == 1 && !s->mapped() && s->plan.kernel == 1 && k3_eligible(s);
}

// Collocation on mapped cells likewise (kernel 0: the sweep kernel).
inline bool k3m_used(const hd_solver *s) {
  return s->quad == 0 && s->mapped() && s->plan.kernel == 1 && k3_eligible(s);
}

// Gauss-Legendre quadrature on mapped cells likewise (kernel 0: the sweep
// kernel).
inline bool k3mg_used(const hd_solver *s) {
  return s->quad == 1 && s->mapped() && s->plan.kernel == 1 && k3_eligible(s);
}

// The dimension-split passes (plan kernel 2, stage_split.h) cover d = 6
// (3 x + 3 v) and d = 5 (3 x + 2 v) at degrees 4 and 5, Gauss-Lobatto
// collocation on Cartesian cells.
inline bool split_eligible(const hd_solver *s) {
  return (s->n == 5 || s->n == 6) && s->quad == 0 && !s->mapped() && s->dx == 3 &&
         (s->d == 6 || s->d == 5);
}
inline bool split_used(const hd_solver *s) { return s->plan.kernel == 2 && split_eligible(s); }

// Grid, workgroup size and dynamic LDS of one stage launch under the
// solver's plan (for plan kernel 2 its first pass).
hd::LaunchShape shape_of(const hd_solver *s);

// Entries and launch shapes of the two passes of plan kernel 2.
struct SplitShapes {
  hd::SplitEntry e;
  hd::LaunchShape x, v;
};
SplitShapes split_shapes(const hd_solver *s);

// The stage kernel of the solver's plan; k3_role selects the 6D degree-3
// kernel's variant (0 general, 1 first stage, 2 late increment); list != 0
// its work-list form (stage_list_kernel / stage_k3_list_kernel; only for
// solves with list_capable), nullptr if none is compiled.
const void *stage_entry(const hd_solver *s, int k3_role = 0, int list = 0);

// The stages of s run the generic kernel or the 6D degree-3 collocation
// kernel on Cartesian cells with a prescribed field: kernels with a
// work-list form. (The Gauss-Legendre and mapped-cell kernels take a second
// table argument, the Vlasov-Poisson field adds per-solve launches, and the
// dimension-split plan takes two launches per stage.)
inline bool list_capable(const hd_solver *s) {
  return s->quad == 0 && !s->mapped() && s->field_kind != 2 && s->plan.kernel != 2;
}

// Kernel parameters, launch shape and 6D degree-3 role of one operator
// application (mode 0: out = L(in)) or fused RK stage (mode 1: in -> u_out,
// increment in the workspace) of s: exactly what its own launch uses.
template <typename P>
void fill_stage(const hd_solver *s, const double *in, void *out, double *u_out, int mode, int stage,
                double dt, StageParams<P> *prm, LaunchShape *ls, int *k3_role);

// Enqueue stage `stage` of one RK step of s on st, from solution buffer par
// to 1 - par (as enqueue_step does for each of its five stages).
hd_status enqueue_stage_of(hd_solver *s, int par, int stage, double dt, hipStream_t st);

// Let kernel fn use up to 160 KiB of LDS minus its static LDS (once per entry).
hipError_t allow_large_lds(const void *fn);

// Enqueue the five fused stages of one RK step of s on st, starting from
// solution buffer `par` (the solution ends in buffer 1 - par). s->cur is
// not changed.
hd_status enqueue_step(hd_solver *s, int par, double dt, hipStream_t st);

// Vlasov-Poisson field (hd_vp.hip): modes per dimension at most
// kVpMaxModes; workspace layout from `off` (returns the end offset); upload
// of the field matrices; enqueue of the field of state u into the E table.
constexpr int kVpMaxModes = 16;
size_t vp_layout(hd_solver *s, size_t off);
hd_status vp_upload(hd_solver *s);
// moments = true: the density from the stage kernel's velocity moments of u
// (valid only when s->vp_mom_src == u), else from u itself.
hd_status vp_enqueue(hd_solver *s, const double *u, hipStream_t st, bool moments = false);

// Kernel parameters of a solver (everything but the per-launch fields:
// buffers, mode, RK coefficients, dt). kernel = 1 passes constant fields in
// the phase-space form the specialised kernel reads.
template <typename P>
void fill_params(const hd_solver *s, StageParams<P> *prm, int kernel) {
  std::memset(prm, 0, sizeof(*prm));
  prm->ncells = (unsigned)s->ncells;
  unsigned st = 1;
  for (int j = 0; j < s->d; ++j) {
    prm->cells[j] = (unsigned)s->mesh.cells[j];
    prm->cstride[j] = st;
    st *= (unsigned)s->mesh.cells[j];
    prm->inv_h[j] = (P)(1.0 / s->h[j]);
    // lift = 1 / w_0 = 1 / w_k (boundary Gauss-Lobatto weight on [0,1]).
    prm->lift_inv_h[j] = (P)(1.0 / (s->tab.w[0] * s->h[j]));
    prm->a_const[j] = (P)s->a_const[j];
    prm->vlo[j] = (P)s->mesh.lo[j];
    prm->vh[j] = (P)s->h[j];
  }
  for (int m = 0; m < s->n; ++m) prm->xi[m] = (P)s->tab.xi[m];
  for (int m = 0; m < s->n; ++m) prm->gw[m] = s->tab.w[m];
  for (int q = 0; q < s->n * s->n; ++q) prm->Dm[q] = (P)s->tab.D[q];
  // The Vlasov-Poisson field (kind 2) is a phase-space field whose E table
  // is recomputed before each stage.
  prm->field_kind = s->field_kind == 0 ? 0 : 1;
  prm->esign = (P)s->esign;
  prm->E = reinterpret_cast<const P *>(s->E());
  prm->xcd_remap = s->plan.xcd_remap;
  prm->cells_per_wg = (unsigned)s->plan.cells_per_wg;
  if (kernel == 1 && s->field_kind == 0) {
    // The specialised kernel reads every field in phase-space form: the
    // constant a_x as a velocity coordinate with zero cell width, the
    // constant a_v from the E table (filled with the constants).
    for (int j = 0; j < s->dx; ++j) {
      prm->vlo[s->dx + j] = (P)s->a_const[j];
      prm->vh[s->dx + j] = P(0);
    }
    prm->esign = P(1);
  }
}

}  // namespace rt
}  // namespace hd
