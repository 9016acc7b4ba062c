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

// Gauss-Legendre variant (Sec. 2.5, the paper's default quadrature): n = k+1
// points g_q with weights om_q on [0,1], and the matrices that move between
// the GL nodal basis and values at the points.
struct GaussTables1D {
  int n = 0;
  double g[8] = {0}, om[8] = {0};
  double B[64] = {0};     // B[q * n + i] = l_i(g_q)
  double Binv[64] = {0};  // B^{-1}
  double Dg[64] = {0};    // derivative at g_q of the interpolant through the points
  double ext[2][8] = {};  // ext[s][q] = Binv[s * k][q]: the trace at xi = s
  double lift[2][8] = {}; // ext[s][q] / om_q
};

// Number of eigenvalues below x of the symmetric tridiagonal Jacobi matrix of
// the Legendre polynomials on [-1,1] (zero diagonal, off-diagonal
// m / sqrt(4 m^2 - 1)), by the Sturm sequence of its leading minors.
inline int legendre_jacobi_count_below(int n, long double x) {
  int count = 0;
  long double q = -x;  // d_1 = a_1 - x with a_1 = 0
  for (int i = 0;; ++i) {
    if (q < 0) ++count;
    if (i + 1 == n) break;
    const long double m = (long double)(i + 1);
    const long double b2 = m * m / (4.0L * m * m - 1.0L);
    long double qq = q == 0.0L ? 1e-30L : q;
    q = -x - b2 / qq;
  }
  return count;
}

inline bool make_gauss_tables(const Tables1D &gl, GaussTables1D *t) {
  const int n = gl.n, k = n - 1;
  if (n < 2 || n > 8) return false;
  t->n = n;
  // Points: the eigenvalues of the Jacobi matrix, one bisection per index.
  long double s[8];
  for (int m = 0; m < n; ++m) {
    long double lo = -1.0L, hi = 1.0L;
    for (int it = 0; it < 90; ++it) {
      const long double mid = 0.5L * (lo + hi);
      if (legendre_jacobi_count_below(n, mid) > m) hi = mid;
      else lo = mid;
    }
    s[m] = 0.5L * (lo + hi);
  }
  long double g[8];
  for (int m = 0; m < n; ++m) g[m] = 0.5L * (1.0L + s[m]);
  // Weights from the moment conditions sum_m om_m g_m^p = 1/(p+1), p < n.
  long double A[8][9];
  for (int p = 0; p < n; ++p) {
    for (int m = 0; m < n; ++m) A[p][m] = powl(g[m], p);
    A[p][n] = 1.0L / (p + 1);
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
    for (int c = 0; c <= n; ++c) {
      const long double tmp = A[col][c];
      A[col][c] = A[piv][c];
      A[piv][c] = tmp;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const long double f = A[r][col] / A[col][col];
      for (int c = col; c <= n; ++c) A[r][c] -= f * A[col][c];
    }
  }
  long double om[8];
  for (int m = 0; m < n; ++m) om[m] = A[m][n] / A[m][m];
  // Lagrange values and derivatives of the GL basis at the points (for even
  // k the midpoint is both a point and a node, so no division by x - xi_r):
  // l_i(x) = prod_{r != i} (x - xi_r) / (xi_i - xi_r),
  // l_i'(x) = sum_{s != i} 1 / (xi_i - xi_s) prod_{r != i, s} (x - xi_r) / (xi_i - xi_r).
  long double B[8][8], DB[8][8];
  for (int q = 0; q < n; ++q)
    for (int i = 0; i < n; ++i) {
      const long double xq = g[q], xii = (long double)gl.xi[i];
      long double v = 1.0L, dsum = 0.0L;
      for (int r = 0; r < n; ++r)
        if (r != i) v *= (xq - (long double)gl.xi[r]) / (xii - (long double)gl.xi[r]);
      for (int sx = 0; sx < n; ++sx) {
        if (sx == i) continue;
        long double tm = 1.0L / (xii - (long double)gl.xi[sx]);
        for (int r = 0; r < n; ++r)
          if (r != i && r != sx) tm *= (xq - (long double)gl.xi[r]) / (xii - (long double)gl.xi[r]);
        dsum += tm;
      }
      B[q][i] = v;
      DB[q][i] = dsum;
    }
  // B^{-1} by Gauss-Jordan elimination with partial pivoting.
  long double T[8][16];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) T[r][c] = c < n ? B[r][c] : (c - n == r ? 1.0L : 0.0L);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(T[r][col]) > fabsl(T[piv][col])) piv = r;
    if (T[piv][col] == 0.0L) return false;
    for (int c = 0; c < 2 * n; ++c) {
      const long double tmp = T[col][c];
      T[col][c] = T[piv][c];
      T[piv][c] = tmp;
    }
    const long double inv = 1.0L / T[col][col];
    for (int c = 0; c < 2 * n; ++c) T[col][c] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const long double f = T[r][col];
      for (int c = 0; c < 2 * n; ++c) T[r][c] -= f * T[col][c];
    }
  }
  for (int q = 0; q < n; ++q) {
    t->g[q] = (double)g[q];
    t->om[q] = (double)om[q];
    for (int i = 0; i < n; ++i) {
      t->B[q * n + i] = (double)B[q][i];
      t->Binv[q * n + i] = (double)T[q][n + i];
      long double dg = 0.0L;  // Dg = DB B^{-1}
      for (int m = 0; m < n; ++m) dg += DB[q][m] * T[m][n + i];
      t->Dg[q * n + i] = (double)dg;
    }
  }
  for (int sd = 0; sd < 2; ++sd)
    for (int q = 0; q < n; ++q) {
      const long double e = T[sd * k][n + q];
      t->ext[sd][q] = (double)e;
      t->lift[sd][q] = (double)(e / om[q]);
    }
  return true;
}

// The collocation rule in the same form (the points are the nodes): B =
// B^{-1} = I, Dg = D, ext[s] = e_{s k}, lift[s][q] = delta_{q, s k} / w_q,
// for the kernel that evaluates mapped cells with either rule.
inline void make_gl_quad_tables(const Tables1D &gl, GaussTables1D *t) {
  const int n = gl.n, k = n - 1;
  *t = GaussTables1D{};
  t->n = n;
  for (int q = 0; q < n; ++q) {
    t->g[q] = gl.xi[q];
    t->om[q] = gl.w[q];
    for (int i = 0; i < n; ++i) {
      t->B[q * n + i] = q == i ? 1.0 : 0.0;
      t->Binv[q * n + i] = q == i ? 1.0 : 0.0;
      t->Dg[q * n + i] = gl.D[q * n + i];
    }
  }
  for (int sd = 0; sd < 2; ++sd) {
    t->ext[sd][sd * k] = 1.0;
    t->lift[sd][sd * k] = 1.0 / gl.w[sd * k];
  }
}

}  // namespace hd
