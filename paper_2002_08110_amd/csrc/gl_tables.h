// Host-side 1D tables of the library: Gauss-Lobatto points and weights on
// [0,1] and the nodal differentiation matrix (Sec. 2.3 nodes, Sec. 2.5
// quadrature). Computed in long double.
#pragma once

#include <cmath>

namespace hd {

struct Tables1D {
  int n = 0;
  double xi[8] = {0};
  double w[8] = {0};
  double D[64] = {0};  // D[q * n + m] = l'_m(xi_q)
};

// Interior Gauss-Lobatto points are the roots of the Jacobi polynomial
// P^{(1,1)}_{k-1} (P'_k is proportional to it). Three-term recurrence:
// n(n+2)/(n+1) P_n = (2n+1) x P_{n-1} - n P_{n-2}, P_0 = 1, P_1 = 2x;
// the derivative follows by differentiating the recurrence.
inline void jacobi11(int deg, long double x, long double *p, long double *dp) {
  long double pm2 = 1.0L, dpm2 = 0.0L;
  if (deg == 0) {
    *p = 1.0L;
    *dp = 0.0L;
    return;
  }
  long double pm1 = 2.0L * x, dpm1 = 2.0L;
  for (int n = 2; n <= deg; ++n) {
    const long double c = (long double)(n + 1) / ((long double)n * (n + 2));
    const long double pn = c * ((2 * n + 1) * x * pm1 - n * pm2);
    const long double dpn = c * ((2 * n + 1) * (pm1 + x * dpm1) - n * dpm2);
    pm2 = pm1;
    dpm2 = dpm1;
    pm1 = pn;
    dpm1 = dpn;
  }
  *p = pm1;
  *dp = dpm1;
}

inline bool make_tables(int k, Tables1D *t) {
  if (k < 1 || k > 7) return false;
  const int n = k + 1;
  t->n = n;
  long double s[8];
  s[0] = -1.0L;
  s[k] = 1.0L;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int m = 1; m < k; ++m) {
    long double x = -cosl(pi * m / k);  // Chebyshev-Gauss-Lobatto start
    for (int it = 0; it < 200; ++it) {
      long double p, dp;
      jacobi11(k - 1, x, &p, &dp);
      const long double dx = p / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    s[m] = x;
  }
  for (int m = 0; m < k; ++m)
    if (!(s[m] < s[m + 1])) return false;  // Newton must land on distinct ordered roots
  long double xi[8];
  for (int m = 0; m <= k; ++m) xi[m] = 0.5L * (1.0L + s[m]);
  xi[0] = 0.0L;
  xi[k] = 1.0L;
  // Weights from the moment conditions sum_m w_m xi_m^p = 1/(p+1),
  // p = 0..k (Vandermonde system, Gaussian elimination with pivoting).
  long double A[8][9];
  for (int p = 0; p <= k; ++p) {
    for (int m = 0; m <= k; ++m) A[p][m] = powl(xi[m], p);
    A[p][n] = 1.0L / (p + 1);
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
    for (int c = 0; c <= n; ++c) {
      long double tmp = A[col][c];
      A[col][c] = A[piv][c];
      A[piv][c] = tmp;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const long double f = A[r][col] / A[col][col];
      for (int c = col; c <= n; ++c) A[r][c] -= f * A[col][c];
    }
  }
  long double w[8];
  for (int m = 0; m < n; ++m) w[m] = A[m][n] / A[m][m];
  // Differentiation matrix from barycentric weights lam_m = 1/prod(xi_m - xi_r):
  // D[q][m] = (lam_m / lam_q) / (xi_q - xi_m) for q != m, rows sum to zero.
  long double lam[8];
  for (int m = 0; m < n; ++m) {
    long double pr = 1.0L;
    for (int r = 0; r < n; ++r)
      if (r != m) pr *= xi[m] - xi[r];
    lam[m] = 1.0L / pr;
  }
  for (int q = 0; q < n; ++q) {
    long double diag = 0.0L;
    for (int m = 0; m < n; ++m) {
      if (m == q) continue;
      const long double v = (lam[m] / lam[q]) / (xi[q] - xi[m]);
      t->D[q * n + m] = (double)v;
      diag -= v;
    }
    t->D[q * n + q] = (double)diag;
  }
  for (int m = 0; m < n; ++m) {
    t->xi[m] = (double)xi[m];
    t->w[m] = (double)w[m];
  }
  return true;
}

}  // namespace hd
