// Host check of the even-odd line transforms of the Gauss-Legendre sweep
// kernel (csrc/stage_gauss.h, compiled for the CPU with the device
// stand-in of tests/native/emu): for random centro-symmetric and
// centro-antisymmetric matrices of every size 2..6 and for the library's own
// interpolation and derivative tables (B, B^-1, Dg for degrees 1..5), the
// even-odd product equals the dense product to rounding, and the tables have
// the symmetry the even-odd form assumes. Prints one line per case; exit
// status 1 on the first failure.
#include "hip/hip_runtime.h"

#include <cmath>
#include <cstdio>
#include <random>

#include "gl_tables.h"
#include "stage_gauss.h"

thread_local emu_dim3 threadIdx, blockIdx;
emu_dim3 blockDim, gridDim;
void emu_syncthreads() {}
int emu_mov_dpp(int v, int) { return v; }
namespace hd {
alignas(256) unsigned char smem_raw[16];
}

namespace {

std::mt19937_64 rng(2002);

template <int N, bool ANTI>
bool check(const double *M, const char *what, int k) {
  hd::GaussEvenOdd<N, double> c;
  hd::gauss_eo_make<N, ANTI>(M, c);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double worst = 0.0;
  for (int rep = 0; rep < 200; ++rep) {
    double v[N], w[N];
    for (int m = 0; m < N; ++m) v[m] = w[m] = U(rng);
    hd::gauss_eo_apply<N, ANTI>(c, w);
    double scale = 0.0;
    for (int q = 0; q < N; ++q)
      for (int m = 0; m < N; ++m) scale += std::fabs(M[q * N + m] * v[m]);
    for (int q = 0; q < N; ++q) {
      double d = 0.0;
      for (int m = 0; m < N; ++m) d += M[q * N + m] * v[m];
      worst = std::fmax(worst, std::fabs(w[q] - d) / scale);
    }
  }
  const bool ok = worst <= 1e-14;
  std::printf("%s k=%d N=%d %s: max |even-odd - dense| / sum |terms| = %.2e %s\n", what, k, N,
              ANTI ? "antisymmetric" : "symmetric", worst, ok ? "ok" : "FAIL");
  return ok;
}

// Deviation of M from (anti)symmetry under q, m -> N-1-q, N-1-m.
double asym(const double *M, int n, bool anti) {
  double worst = 0.0, scale = 0.0;
  for (int q = 0; q < n * n; ++q) scale = std::fmax(scale, std::fabs(M[q]));
  for (int q = 0; q < n; ++q)
    for (int m = 0; m < n; ++m) {
      const double mirror = M[(n - 1 - q) * n + (n - 1 - m)];
      worst = std::fmax(worst, std::fabs(M[q * n + m] - (anti ? -mirror : mirror)));
    }
  return worst / scale;
}

template <int N>
bool random_cases() {
  std::uniform_real_distribution<double> U(-2.0, 2.0);
  double S[N * N], A[N * N];
  for (int q = 0; q < N; ++q)
    for (int m = 0; m < N; ++m) {
      const int q2 = N - 1 - q, m2 = N - 1 - m;
      if (q * N + m < q2 * N + m2) {
        S[q * N + m] = S[q2 * N + m2] = U(rng);
        A[q * N + m] = U(rng);
        A[q2 * N + m2] = -A[q * N + m];
      } else if (q * N + m == q2 * N + m2) {
        S[q * N + m] = U(rng);
        A[q * N + m] = 0.0;  // the centre of odd N
      }
    }
  return check<N, false>(S, "random", 0) && check<N, true>(A, "random", 0);
}

template <int N>
bool table_cases() {
  hd::Tables1D t;
  hd::GaussTables1D g;
  if (!hd::make_tables(N - 1, &t) || !hd::make_gauss_tables(t, &g)) return false;
  const double sb = asym(g.B, N, false), sbi = asym(g.Binv, N, false), sd = asym(g.Dg, N, true);
  double DgT[N * N];
  for (int q = 0; q < N; ++q)
    for (int m = 0; m < N; ++m) DgT[q * N + m] = g.Dg[m * N + q];
  std::printf("tables k=%d: asymmetry B %.1e, B^-1 %.1e, Dg %.1e (antisymmetric)\n", N - 1, sb, sbi, sd);
  return sb <= 1e-14 && sbi <= 1e-13 && sd <= 1e-13 && check<N, false>(g.B, "B", N - 1) &&
         check<N, false>(g.Binv, "B^-1", N - 1) && check<N, true>(g.Dg, "Dg", N - 1) &&
         check<N, true>(DgT, "Dg^T", N - 1);
}

}  // namespace

int main() {
  bool ok = random_cases<2>() && random_cases<3>() && random_cases<4>() && random_cases<5>() &&
            random_cases<6>();
  ok = ok && table_cases<2>() && table_cases<3>() && table_cases<4>() && table_cases<5>() &&
       table_cases<6>();
  std::printf("%s\n", ok ? "all ok" : "FAILED");
  return ok ? 0 : 1;
}
