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
  // Workspace layout (offsets into the caller's buffer).
  size_t off_u[2] = {0, 0}, off_du = 0, off_E = 0, off_part = 0, total = 0;
  char *ws = nullptr;
  int cur = 0;  // which of the two solution buffers holds the solution
  hd_plan plan{};
  // Captured RK steps (index = solution buffer parity at the start).
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  double gdt = 0.0;
  bool gvalid = false;
  uint64_t version = 0;  // bumped when the plan, field or memory changes

  double *u(int i) const { return reinterpret_cast<double *>(ws + off_u[i]); }
  void *du() const { return ws + off_du; }
  void *E() const { return ws + off_E; }
  double *part() const { return reinterpret_cast<double *>(ws + off_part); }
  size_t psize() const { return prec == HD_FP32 ? sizeof(float) : sizeof(double); }
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

// Grid, workgroup size and dynamic LDS of one stage launch under the
// solver's plan.
hd::LaunchShape shape_of(const hd_solver *s);

// Entry of the compiled stage kernel of the solver's plan; nullptr if none
// is compiled.
const void *stage_entry(const hd_solver *s);

// Enqueue the five fused stages of one RK step of s on st, starting from
// solution buffer `par` (the solution ends in buffer 1 - par). s->cur is
// not changed.
hd_status enqueue_step(hd_solver *s, int par, double dt, hipStream_t st);

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
  for (int q = 0; q < s->n * s->n; ++q) prm->Dm[q] = (P)s->tab.D[q];
  prm->field_kind = s->field_kind;
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
