// Vlasov-Poisson field (Sec. 6): electrons on a neutralizing background,
//   rho(x) = int f dv,  -Laplace phi = 1 - rho,  E = -grad phi,  a = (v, -E),
// recomputed from the input of every RK stage and written into the E table
// that the stage kernels read (x-points p = xcell * n^dx + xnode).
//
// Steps, all FP64 and deterministic (fixed summation order):
//  1. density: rho(x_p) = sum over v-cells and v-nodes of the GL weight times
//     f, in two passes (partial sums over groups of v-cells, then the groups
//     in order);
//  2. the weighted density rho_p W_p / |Omega_x| gathered into a tensor over
//     the 1D x-point sets of each dimension (x_{j,a} = lo_j + (c + xi_i) h_j);
//  3. rho_hat_m = sum_p W_p rho_p exp(-i k_m.x_p) / |Omega_x| for the modes
//     m in [-M, M]^dx, computed dimension by dimension (the exponential
//     factorizes over dimensions);
//  4. E_hat_j = i k_j rho_hat / |k|^2 (zero for m = 0, which the background
//     balances);
//  5. E_j(x_p) = sum_m Re[E_hat_j exp(i k_m.x_p)], again dimension by
//     dimension, and the real part stored in the E table.
// The same field as a direct double sum over points and modes, up to the
// order of rounding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "hd_internal.h"

namespace hd {
namespace {

constexpr int kVpThreads = 256;

struct VpGeom {
  int dx, n, M;
  int X[3], K[3];            // points and modes per x-dim (1 for absent dims)
  int cells[3];
  long long nxc, nxn, nvc, nvn, nd, npts;
  int groups;
  double hv, vol;
  double h[3], w[8];
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Pass 1 of the density: partial[g][p] = sum over the v-cells of group g and
// r < R of wts[r] * src[cell * cstride + xnode + nxn * r]. From the state:
// cstride = n^d, R = all v-nodes, wts = products of the velocity GL weights.
// From the stage kernel's moments (already summed over the last two
// velocity dimensions): cstride = 256, R = n (the first velocity node), wts =
// the GL weights.
__global__ void vp_density_partial(VpGeom g, const double *__restrict__ src, long long cstride,
                                   int R, const double *__restrict__ wts,
                                   double *__restrict__ partial) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.npts * g.groups) return;
  const long long p = idx % g.npts, grp = idx / g.npts;
  const long long xc = p / g.nxn, xn = p % g.nxn;
  const long long c0 = grp * g.nvc / g.groups, c1 = (grp + 1) * g.nvc / g.groups;
  double s = 0.0;
  for (long long cv = c0; cv < c1; ++cv) {
    const double *cellu = src + (xc + g.nxc * cv) * cstride + xn;
    for (int r = 0; r < R; ++r) s += wts[r] * cellu[g.nxn * r];
  }
  partial[grp * g.npts + p] = s;
}

// Pass 2: rho_p = (prod h_v) sum_groups partial (in group order), then the
// weighted density into the tensor T[p1 + X1 (p2 + X2 p3)].
__global__ void vp_density_final(VpGeom g, const double *__restrict__ partial,
                                 double2 *__restrict__ T) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.npts) return;
  double s = 0.0;
  for (int grp = 0; grp < g.groups; ++grp) s += partial[(long long)grp * g.npts + p];
  const double rho = g.hv * s;
  long long xc = p / g.nxn, xn = p % g.nxn, t = 0, stride = 1;
  double W = 1.0;
  for (int j = 0; j < g.dx; ++j) {
    const int c = (int)(xc % g.cells[j]), i = (int)(xn % g.n);
    xc /= g.cells[j];
    xn /= g.n;
    W *= g.h[j] * g.w[i];
    t += (long long)(c * g.n + i) * stride;
    stride *= g.X[j];
  }
  T[t] = make_double2(W * rho / g.vol, 0.0);
}

// out[o][m][i] = sum_a mat[m][a] in[o][a][i] (complex): one transform along
// the middle axis of a 3-index array.
__global__ void vp_axis(const double2 *__restrict__ in, double2 *__restrict__ out,
                        const double2 *__restrict__ mat, long long O, int A, int Mo, long long I) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= O * Mo * I) return;
  const long long i = idx % I, r = idx / I;
  const int m = (int)(r % Mo);
  const long long o = r / Mo;
  double2 s = make_double2(0.0, 0.0);
  for (int a = 0; a < A; ++a) {
    const double2 v = cmul(mat[(long long)m * A + a], in[(o * A + a) * I + i]);
    s.x += v.x;
    s.y += v.y;
  }
  out[idx] = s;
}

// E_hat_j[m] = i k_j rho_hat[m] / |k|^2, k_j = kf_j (m_j - M); zero mode: 0.
__global__ void vp_spectrum(VpGeom g, const double2 *__restrict__ rhat, double2 *__restrict__ Eh,
                            double kf0, double kf1, double kf2) {
  const long long nm = (long long)g.K[0] * g.K[1] * g.K[2];
  const long long mi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= nm) return;
  const double kf[3] = {kf0, kf1, kf2};
  double kv[3] = {0.0, 0.0, 0.0}, k2 = 0.0;
  long long r = mi;
  for (int j = 0; j < g.dx; ++j) {
    const int m = (int)(r % g.K[j]) - g.M;
    r /= g.K[j];
    kv[j] = kf[j] * m;
    k2 += kv[j] * kv[j];
  }
  const double2 rh = rhat[mi];
  for (int j = 0; j < g.dx; ++j) {
    const double c = k2 > 0.0 ? kv[j] / k2 : 0.0;
    Eh[j * nm + mi] = make_double2(-c * rh.y, c * rh.x);
  }
}

// E table entry of x-point p, component j: the real part of R[t(p)].
template <typename P>
__global__ void vp_scatter(VpGeom g, const double2 *__restrict__ R, int j, P *__restrict__ E) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.npts) return;
  long long xc = p / g.nxn, xn = p % g.nxn, t = 0, stride = 1;
  for (int m = 0; m < g.dx; ++m) {
    const int c = (int)(xc % g.cells[m]), i = (int)(xn % g.n);
    xc /= g.cells[m];
    xn /= g.n;
    t += (long long)(c * g.n + i) * stride;
    stride *= g.X[m];
  }
  E[p * g.dx + j] = (P)R[t].x;
}

unsigned blocks_for(long long n) { return (unsigned)((n + kVpThreads - 1) / kVpThreads); }

VpGeom geom_of(const hd_solver *s) {
  VpGeom g{};
  g.dx = s->dx;
  g.n = s->n;
  g.M = s->vp_modes;
  g.nxc = g.nxn = g.nvc = g.nvn = 1;
  for (int j = 0; j < 3; ++j) {
    g.X[j] = 1;
    g.K[j] = 1;
    g.cells[j] = 1;
    g.h[j] = 1.0;
  }
  g.vol = 1.0;
  g.hv = 1.0;
  for (int j = 0; j < s->dx; ++j) {
    g.cells[j] = s->mesh.cells[j];
    g.X[j] = s->mesh.cells[j] * s->n;
    g.K[j] = 2 * s->vp_modes + 1;
    g.h[j] = s->h[j];
    g.nxc *= s->mesh.cells[j];
    g.nxn *= s->n;
    g.vol *= s->mesh.hi[j] - s->mesh.lo[j];
  }
  for (int j = s->dx; j < s->d; ++j) {
    g.nvc *= s->mesh.cells[j];
    g.nvn *= s->n;
    g.hv *= s->h[j];
  }
  for (int i = 0; i < s->n; ++i) g.w[i] = s->tab.w[i];
  g.nd = s->nd;
  g.npts = g.nxc * g.nxn;
  g.groups = s->vp_groups;
  return g;
}

}  // namespace

namespace rt {

// Lay out the Vlasov-Poisson scratch (phase-space meshes only) from byte
// offset `off` of the workspace; returns the end offset. Sized for up to
// kVpMaxModes modes per dimension.
size_t vp_layout(hd_solver *s, size_t off) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  s->vp_groups = 0;
  if (s->dx != s->dv) return off;
  long long npts = 1, nvc = 1, nvn = 1, big = 1, mats = 0, nm = 1;
  for (int j = 0; j < s->dx; ++j) {
    const long long X = (long long)s->mesh.cells[j] * s->n, K = 2 * kVpMaxModes + 1;
    npts *= X;
    big *= std::max(X, K);
    mats += 2 * K * X;
    nm *= K;
  }
  for (int j = s->dx; j < s->d; ++j) {
    nvc *= s->mesh.cells[j];
    nvn *= s->n;
  }
  // partial sums over enough v-cell groups for ~2^20 threads
  const long long g = std::max(1LL, std::min(nvc, (1LL << 20) / std::max(1LL, npts)));
  s->vp_groups = (int)g;
  s->off_vp_partial = off;
  off = up(off + (size_t)(g * npts) * sizeof(double));
  s->off_vp_wv = off;
  off = up(off + (size_t)(nvn + s->n) * sizeof(double));
  s->off_vp_A = off;
  off = up(off + (size_t)big * sizeof(double2));
  s->off_vp_B = off;
  off = up(off + (size_t)big * sizeof(double2));
  s->off_vp_Eh = off;
  off = up(off + (size_t)(s->dx * nm) * sizeof(double2));
  s->off_vp_mats = off;
  off = up(off + (size_t)mats * sizeof(double2));
  // one moment per thread and cell of the 6D degree-3 kernel
  s->vp_mom_bytes = k3_eligible(s) ? (size_t)s->ncells * 256 * sizeof(double) : 0;
  s->off_vp_mom = off;
  off = up(off + s->vp_mom_bytes);
  return off;
}

// Field matrices of the current modes and the velocity weights, uploaded
// into the Vlasov-Poisson region.
hd_status vp_upload(hd_solver *s) {
  const VpGeom g = geom_of(s);
  std::vector<double> wv((size_t)g.nvn);
  for (long long vn = 0; vn < g.nvn; ++vn) {
    double w = 1.0;
    long long r = vn;
    for (int j = 0; j < s->dv; ++j) {
      w *= s->tab.w[r % s->n];
      r /= s->n;
    }
    wv[(size_t)vn] = w;
  }
  for (int i = 0; i < s->n; ++i) wv.push_back(s->tab.w[i]);
  std::vector<double2> mats;
  for (int j = 0; j < s->dx; ++j) {
    const double kf = 2.0 * M_PI / (s->mesh.hi[j] - s->mesh.lo[j]);
    // forward F[m][a] = exp(-i k_m x_a); inverse G[a][m] = exp(+i k_m x_a)
    std::vector<double> x((size_t)g.X[j]);
    for (int c = 0; c < s->mesh.cells[j]; ++c)
      for (int i = 0; i < s->n; ++i)
        x[(size_t)(c * s->n + i)] = s->mesh.lo[j] + (c + s->tab.xi[i]) * s->h[j];
    for (int m = 0; m < g.K[j]; ++m)
      for (int a = 0; a < g.X[j]; ++a) {
        const double ph = kf * (m - g.M) * x[(size_t)a];
        mats.push_back(make_double2(std::cos(ph), -std::sin(ph)));
      }
    for (int a = 0; a < g.X[j]; ++a)
      for (int m = 0; m < g.K[j]; ++m) {
        const double ph = kf * (m - g.M) * x[(size_t)a];
        mats.push_back(make_double2(std::cos(ph), std::sin(ph)));
      }
  }
  HD_HIP(hipMemcpy(s->vp_wv(), wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice));
  HD_HIP(hipMemcpy(s->vp_mats(), mats.data(), mats.size() * sizeof(double2),
                   hipMemcpyHostToDevice));
  return HD_OK;
}

// Enqueue steps 1-5 for the state `u` on `st`, writing the E table.
hd_status vp_enqueue(hd_solver *s, const double *u, hipStream_t st, bool moments) {
  const VpGeom g = geom_of(s);
  double2 *A = s->vp_bufA(), *B = s->vp_bufB(), *Eh = s->vp_Ehat();
  const double2 *mats = s->vp_mats();
  if (moments && (s->vp_mom_src != u || !s->vp_mom_bytes))
    return fail(HD_ERR_STATE, "velocity moments do not describe this state");
  if (moments)
    hipLaunchKernelGGL(vp_density_partial, dim3(blocks_for(g.npts * g.groups)), dim3(kVpThreads),
                       0, st, g, s->vp_mom(), (long long)g.nxn * s->n, s->n,
                       s->vp_wv() + g.nvn, s->vp_partial());
  else
    hipLaunchKernelGGL(vp_density_partial, dim3(blocks_for(g.npts * g.groups)), dim3(kVpThreads),
                       0, st, g, u, (long long)g.nd, (int)g.nvn, s->vp_wv(), s->vp_partial());
  hipLaunchKernelGGL(vp_density_final, dim3(blocks_for(g.npts)), dim3(kVpThreads), 0, st, g,
                     s->vp_partial(), A);
  // forward: axis 1 (A -> B), axis 2 (B -> A), axis 3 (A -> B); sizes as
  // [outer][axis][inner]
  long long sz[3] = {g.X[0], g.X[1], g.X[2]};
  double2 *in = A, *out = B;
  const double2 *mj = mats;
  const double2 *inv[3];
  for (int j = 0; j < g.dx; ++j) {
    long long O = 1, I = 1;
    for (int q = j + 1; q < 3; ++q) O *= sz[q];
    for (int q = 0; q < j; ++q) I *= sz[q];
    hipLaunchKernelGGL(vp_axis, dim3(blocks_for(O * g.K[j] * I)), dim3(kVpThreads), 0, st, in, out,
                       mj, O, g.X[j], g.K[j], I);
    inv[j] = mj + (long long)g.K[j] * g.X[j];
    mj += 2LL * g.K[j] * g.X[j];
    sz[j] = g.K[j];
    double2 *t = in;
    in = out;
    out = t;
  }
  // `in` holds rho_hat [m3][m2][m1]
  const double kf0 = 2.0 * M_PI / (s->mesh.hi[0] - s->mesh.lo[0]);
  const double kf1 = s->dx > 1 ? 2.0 * M_PI / (s->mesh.hi[1] - s->mesh.lo[1]) : 0.0;
  const double kf2 = s->dx > 2 ? 2.0 * M_PI / (s->mesh.hi[2] - s->mesh.lo[2]) : 0.0;
  const long long nm = (long long)g.K[0] * g.K[1] * g.K[2];
  hipLaunchKernelGGL(vp_spectrum, dim3(blocks_for(nm)), dim3(kVpThreads), 0, st, g, in, Eh, kf0,
                     kf1, kf2);
  // inverse per component: axis 1 (Eh_j -> A), axis 2 (A -> B), axis 3 (B -> A)
  for (int c = 0; c < g.dx; ++c) {
    long long s2[3] = {g.K[0], g.K[1], g.K[2]};
    const double2 *src = Eh + c * nm;
    double2 *dst = A, *other = B;
    for (int j = 0; j < g.dx; ++j) {
      long long O = 1, I = 1;
      for (int q = j + 1; q < 3; ++q) O *= s2[q];
      for (int q = 0; q < j; ++q) I *= s2[q];
      hipLaunchKernelGGL(vp_axis, dim3(blocks_for(O * g.X[j] * I)), dim3(kVpThreads), 0, st, src,
                         dst, inv[j], O, g.K[j], g.X[j], I);
      s2[j] = g.X[j];
      src = dst;
      double2 *t = dst;
      dst = other;
      other = t;
    }
    if (s->prec == HD_FP32_OP_FP64_ACC)
      hipLaunchKernelGGL(vp_scatter<float>, dim3(blocks_for(g.npts)), dim3(kVpThreads), 0, st, g,
                         src, c, reinterpret_cast<float *>(s->E()));
    else
      hipLaunchKernelGGL(vp_scatter<double>, dim3(blocks_for(g.npts)), dim3(kVpThreads), 0, st, g,
                         src, c, reinterpret_cast<double *>(s->E()));
  }
  HD_HIP(hipGetLastError());
  return HD_OK;
}

}  // namespace rt
}  // namespace hd
