/*
 * Plain CPU oracle of the upwind Gauss-Lobatto-collocation DG advection
 * operator and its low-storage Runge-Kutta integrator. TEST INFRASTRUCTURE
 * ONLY: used by tests/, the smoke check and the benchmark's CPU baseline,
 * never by the product library. It is deliberately slow: it evaluates the
 * d-dimensional basis functions and their gradients directly at the
 * quadrature points and forms the weak-form sums as written, with no sum
 * factorization. See oracle.h for the paper passages each part follows.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 6
#define OR_MAXK 8
#define OR_MAXN (OR_MAXK + 1)

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* 1D Gauss-Lobatto rule (Sec. 2.3 nodes, Sec. 2.5 quadrature)              */
/* ------------------------------------------------------------------------ */

/* Legendre P_k(s) and P_k'(s) from the three-term recurrence
 * m P_m = (2m-1) s P_{m-1} - (m-1) P_{m-2} and P_m' = s P_{m-1}' + m P_{m-1}. */
static void legendre(int k, double s, double *p, double *dp) {
  double pm1 = 1.0, dpm1 = 0.0; /* P_0, P_0' */
  double pm = s, dpm = 1.0;     /* P_1, P_1' */
  if (k == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int m = 2; m <= k; ++m) {
    double pn = ((2.0 * m - 1.0) * s * pm - (m - 1.0) * pm1) / m;
    double dpn = s * dpm + m * pm;
    pm1 = pm;
    dpm1 = dpm;
    pm = pn;
    dpm = dpn;
  }
  (void)dpm1;
  *p = pm;
  *dp = dpm;
}

int or_gl_rule(int k, double *xi, double *w) {
  if (k < 1 || k > 16) return -1;
  /* Interior points: roots of P_k' on (-1,1), by Newton's method started at
   * the Chebyshev-Gauss-Lobatto points; P_k'' from Legendre's equation
   * (1-s^2) P'' = 2 s P' - k(k+1) P. */
  double s[17];
  s[0] = -1.0;
  s[k] = 1.0;
  for (int m = 1; m < k; ++m) {
    double x = -cos(OR_PI * m / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, x, &p, &dp);
      double ddp = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / ddp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    s[m] = x;
  }
  /* Weights on [-1,1]: 2 / (k(k+1) P_k(s_m)^2); halved for [0,1]. */
  for (int m = 0; m <= k; ++m) {
    double p, dp;
    legendre(k, s[m], &p, &dp);
    xi[m] = 0.5 * (1.0 + s[m]);
    w[m] = 1.0 / (k * (k + 1.0) * p * p);
  }
  xi[0] = 0.0;
  xi[k] = 1.0;
  return 0;
}

/* 1D Gauss-Legendre rule with k+1 points on [0,1] (the quadrature the paper
 * uses by default, Sec. 2.5 and 5.1): the roots s of P_{k+1}, by Newton's
 * method from the estimates -cos(pi (m + 3/4) / (n + 1/2)), and the weights
 * 2 / ((1 - s^2) P_{k+1}'(s)^2) on [-1,1], halved for [0,1]. */
int or_gauss_rule(int k, double *g, double *w) {
  if (k < 1 || k > 16) return -1;
  const int n = k + 1;
  for (int m = 0; m < n; ++m) {
    double x = -cos(OR_PI * (m + 0.75) / (n + 0.5));
    double p = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, &p, &dp);
      double dx = p / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    legendre(n, x, &p, &dp);
    g[m] = 0.5 * (1.0 + x);
    w[m] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  return 0;
}

/* l_m(x) = prod_{r != m} (x - xi_r) / (xi_m - xi_r). */
double or_lagrange(int k, const double *xi, int m, double x) {
  double v = 1.0;
  for (int r = 0; r <= k; ++r)
    if (r != m) v *= (x - xi[r]) / (xi[m] - xi[r]);
  return v;
}

/* l_m'(x) = sum_{s != m} 1/(xi_m - xi_s) prod_{r != m, s} (x - xi_r)/(xi_m - xi_r). */
double or_lagrange_deriv(int k, const double *xi, int m, double x) {
  double sum = 0.0;
  for (int s = 0; s <= k; ++s) {
    if (s == m) continue;
    double t = 1.0 / (xi[m] - xi[s]);
    for (int r = 0; r <= k; ++r)
      if (r != m && r != s) t *= (x - xi[r]) / (xi[m] - xi[r]);
    sum += t;
  }
  return sum;
}

/* ------------------------------------------------------------------------ */
/* Mesh bookkeeping (Sec. 3.1: the cells are pairs of x- and v-cells)        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int d, dx, dv, n, k;
  int64_t nd;     /* nodes per cell, n^d */
  int64_t ncells; /* prod cells */
  int cells[OR_MAXD];
  int64_t cstride[OR_MAXD]; /* cell index stride per dim (dim 1 fastest) */
  int64_t nstride[OR_MAXD]; /* node index stride per dim */
  double lo[OR_MAXD], hi[OR_MAXD], h[OR_MAXD];
  double xi[OR_MAXN], w[OR_MAXN];
  double L[OR_MAXN][OR_MAXN];  /* L[m][q] = l_m(xi_q) */
  double DL[OR_MAXN][OR_MAXN]; /* DL[m][q] = l_m'(xi_q) */
  double M1[OR_MAXN];          /* diagonal of the 1D reference mass matrix */
  /* Gauss-Legendre quadrature (mode 2): points, weights, the GL basis and
   * its derivative at the points, and the 1D mass matrix it integrates
   * exactly, MG[a][b] = sum_q wg_q l_a(g_q) l_b(g_q), with its inverse. */
  double gq[OR_MAXN], wg[OR_MAXN];
  double LG[OR_MAXN][OR_MAXN];  /* LG[m][q] = l_m(g_q) */
  double DLG[OR_MAXN][OR_MAXN]; /* DLG[m][q] = l_m'(g_q) */
  double MG[OR_MAXN][OR_MAXN], MGinv[OR_MAXN][OR_MAXN];
  double Binv[OR_MAXN][OR_MAXN]; /* inverse of B[q][i] = l_i(g_q) */
  double eps;                    /* x-space deformation (0: Cartesian) */
} or_geom;

/* Inverse of the n x n matrix A by Gauss-Jordan elimination with partial
 * pivoting; returns -1 if A is singular. */
static int invert(int n, double A[OR_MAXN][OR_MAXN], double X[OR_MAXN][OR_MAXN]) {
  double T[OR_MAXN][2 * OR_MAXN];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) T[r][c] = c < n ? A[r][c] : (c - n == r ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(T[r][c]) > fabs(T[piv][c])) piv = r;
    if (T[piv][c] == 0.0) return -1;
    for (int q = 0; q < 2 * n; ++q) {
      double t = T[c][q];
      T[c][q] = T[piv][q];
      T[piv][q] = t;
    }
    double inv = 1.0 / T[c][c];
    for (int q = 0; q < 2 * n; ++q) T[c][q] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = T[r][c];
      for (int q = 0; q < 2 * n; ++q) T[r][q] -= f * T[c][q];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) X[r][c] = T[r][n + c];
  return 0;
}

static int setup_geom(const or_mesh *mesh, int k, or_geom *g) {
  if (!mesh) return -1;
  if (mesh->dim_x < 1 || mesh->dim_x > 3 || mesh->dim_v < 1 || mesh->dim_v > 3)
    return -1;
  if (k < 1 || k > OR_MAXK) return -1;
  memset(g, 0, sizeof(*g));
  g->dx = mesh->dim_x;
  g->dv = mesh->dim_v;
  g->d = g->dx + g->dv;
  g->k = k;
  g->n = k + 1;
  g->nd = 1;
  g->ncells = 1;
  for (int j = 0; j < g->d; ++j) {
    if (mesh->cells[j] < 1 || !(mesh->hi[j] > mesh->lo[j])) return -1;
    g->cells[j] = mesh->cells[j];
    g->cstride[j] = g->ncells;
    g->nstride[j] = g->nd;
    g->ncells *= mesh->cells[j];
    g->nd *= g->n;
    g->lo[j] = mesh->lo[j];
    g->hi[j] = mesh->hi[j];
    g->h[j] = (mesh->hi[j] - mesh->lo[j]) / mesh->cells[j];
  }
  if (or_gl_rule(k, g->xi, g->w)) return -1;
  for (int m = 0; m <= k; ++m)
    for (int q = 0; q <= k; ++q) {
      g->L[m][q] = or_lagrange(k, g->xi, m, g->xi[q]);
      g->DL[m][q] = or_lagrange_deriv(k, g->xi, m, g->xi[q]);
    }
  /* 1D reference mass matrix M1[a][b] = sum_q w_q l_a(xi_q) l_b(xi_q). The
   * d-dimensional cell mass matrix with tensor quadrature is the Kronecker
   * product of these (times prod h_j), so it is diagonal exactly when M1
   * is: the collocation property of Sec. 1.3. Refuse to proceed otherwise. */
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= k; ++b) {
      double m = 0.0;
      for (int q = 0; q <= k; ++q) m += g->w[q] * g->L[a][q] * g->L[b][q];
      if (a == b)
        g->M1[a] = m;
      else if (fabs(m) > 1e-14)
        return -1;
    }
  if (or_gauss_rule(k, g->gq, g->wg)) return -1;
  for (int m = 0; m <= k; ++m)
    for (int q = 0; q <= k; ++q) {
      g->LG[m][q] = or_lagrange(k, g->xi, m, g->gq[q]);
      g->DLG[m][q] = or_lagrange_deriv(k, g->xi, m, g->gq[q]);
    }
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= k; ++b) {
      double m = 0.0;
      for (int q = 0; q <= k; ++q) m += g->wg[q] * g->LG[a][q] * g->LG[b][q];
      g->MG[a][b] = m;
    }
  if (invert(g->n, g->MG, g->MGinv)) return -1;
  {
    double Bm[OR_MAXN][OR_MAXN];
    for (int q = 0; q <= k; ++q)
      for (int i = 0; i <= k; ++i) Bm[q][i] = g->LG[i][q];
    if (invert(g->n, Bm, g->Binv)) return -1;
  }
  g->eps = mesh->map_eps;
  if (!(fabs(g->eps) <= 0.05)) return -1;
  return 0;
}

/* The mapping of the box point X (d coordinates; only the first dx change):
 * x_m = X_m + eps L_m prod_k sin(theta_k), theta_k = 2 pi (X_k - lo_k)/L_k,
 * and its derivative Jx[m][k] = dx_m / dX_k for m, k < dx. */
static void map_point(const or_geom *g, const double *X, double *x, double Jx[3][3]) {
  double s[3], c[3];
  for (int k = 0; k < g->dx; ++k) {
    const double L = g->hi[k] - g->lo[k];
    const double th = 2.0 * OR_PI * (X[k] - g->lo[k]) / L;
    s[k] = sin(th);
    c[k] = cos(th);
  }
  for (int m = 0; m < g->d; ++m) x[m] = X[m];
  double prod = 1.0;
  for (int k = 0; k < g->dx; ++k) prod *= s[k];
  for (int m = 0; m < g->dx; ++m) {
    const double Lm = g->hi[m] - g->lo[m];
    x[m] += g->eps * Lm * prod;
    for (int k = 0; k < g->dx; ++k) {
      double p = 1.0;
      for (int r = 0; r < g->dx; ++r) p *= (r == k) ? c[r] : s[r];
      const double Lk = g->hi[k] - g->lo[k];
      Jx[m][k] = (m == k ? 1.0 : 0.0) + g->eps * Lm * (2.0 * OR_PI / Lk) * p;
    }
  }
}

static void cell_multi(const or_geom *g, int64_t c, int *cm) {
  for (int j = 0; j < g->d; ++j) cm[j] = (int)((c / g->cstride[j]) % g->cells[j]);
}
static void node_multi(const or_geom *g, int64_t q, int *qm) {
  for (int j = 0; j < g->d; ++j) qm[j] = (int)((q / g->nstride[j]) % g->n);
}
static int64_t cell_linear(const or_geom *g, const int *cm) {
  int64_t c = 0;
  for (int j = 0; j < g->d; ++j) c += cm[j] * g->cstride[j];
  return c;
}
static int64_t node_linear(const or_geom *g, const int *qm) {
  int64_t q = 0;
  for (int j = 0; j < g->d; ++j) q += qm[j] * g->nstride[j];
  return q;
}

/* Periodic neighbour of cell cm across dim j in direction dir (+1/-1). */
static int64_t neighbour_cell(const or_geom *g, const int *cm, int j, int dir) {
  int nm[OR_MAXD];
  for (int m = 0; m < g->d; ++m) nm[m] = cm[m];
  nm[j] = (cm[j] + dir + g->cells[j]) % g->cells[j];
  return cell_linear(g, nm);
}

/* Physical coordinate of node qm of cell cm in dim j (through the mapping
 * for the configuration dims). */
static double node_coord(const or_geom *g, const int *cm, const int *qm, int j) {
  if (g->eps == 0.0 || j >= g->dx) return g->lo[j] + (cm[j] + g->xi[qm[j]]) * g->h[j];
  double X[OR_MAXD], x[OR_MAXD], Jx[3][3];
  for (int m = 0; m < g->d; ++m) X[m] = g->lo[m] + (cm[m] + g->xi[qm[m]]) * g->h[m];
  map_point(g, X, x, Jx);
  return x[j];
}

/* Advection field component j at node qm of cell cm (Sec. 6.1: v from the
 * velocity node, E from the table at the configuration node). */
static double field_at(const or_geom *g, const or_field *f, const int *cm,
                       const int *qm, int j) {
  if (f->kind == 0) return f->a[j];
  if (j < g->dx) return node_coord(g, cm, qm, g->dx + j);
  int64_t xcell = 0, xs = 1, xnode = 0, ns = 1;
  for (int m = 0; m < g->dx; ++m) {
    xcell += cm[m] * xs;
    xs *= g->cells[m];
    xnode += qm[m] * ns;
    ns *= g->n;
  }
  int64_t nxn = ns;
  return f->sign * f->E[((xcell * nxn) + xnode) * g->dx + (j - g->dx)];
}

static int check_field(const or_geom *g, const or_field *f) {
  if (!f) return -1;
  if (f->kind == 0) return 0;
  if (f->kind == 1) return (g->dx == g->dv && f->E) ? 0 : -1;
  return -1;
}

int64_t or_num_dofs(const or_mesh *mesh, int k) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
  return g.nd * g.ncells;
}

int or_node_coords(const or_mesh *mesh, int k, double *X) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < g.ncells; ++c) {
    int cm[OR_MAXD], qm[OR_MAXD];
    cell_multi(&g, c, cm);
    for (int64_t q = 0; q < g.nd; ++q) {
      node_multi(&g, q, qm);
      for (int j = 0; j < g.d; ++j)
        X[(c * g.nd + q) * g.d + j] = node_coord(&g, cm, qm, j);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The operator M^{-1} A(u) on one cell (Algorithm 2, Sec. 1.3 weak form)   */
/* ------------------------------------------------------------------------ */

/* phi_i at the node qm of the own cell: prod_m l_{i_m}(xi_{q_m}). */
static double phi_at(const or_geom *g, const int *im, const int *qm) {
  double v = 1.0;
  for (int m = 0; m < g->d; ++m) v *= g->L[im[m]][qm[m]];
  return v;
}

/* d/dx_j phi_i at node qm: l'_{i_j}(xi_{q_j}) / h_j * prod_{m != j} l_{i_m}(xi_{q_m}). */
static double dphi_at(const or_geom *g, const int *im, const int *qm, int j) {
  double v = g->DL[im[j]][qm[j]] / g->h[j];
  for (int m = 0; m < g->d; ++m)
    if (m != j) v *= g->L[im[m]][qm[m]];
  return v;
}

/* Volume quadrature weight W_q = prod_j h_j w_{q_j}. */
static double vol_weight(const or_geom *g, const int *qm) {
  double v = 1.0;
  for (int m = 0; m < g->d; ++m) v *= g->h[m] * g->w[qm[m]];
  return v;
}

/* Face quadrature weight on a face normal to dim j: prod_{m != j} h_m w_{q_m}. */
static double face_weight(const or_geom *g, const int *qm, int j) {
  double v = 1.0;
  for (int m = 0; m < g->d; ++m)
    if (m != j) v *= g->h[m] * g->w[qm[m]];
  return v;
}

/* Scratch for one cell evaluation. */
typedef struct {
  double *uh;   /* u_h at the quadrature points of the cell */
  double *rhs;  /* V - F, then divided by the mass diagonal */
  double *acell; /* a_j at each node: acell[q * d + j] */
  int *multi;    /* multi-index of every node: multi[q * d + m] (mode 2) */
} or_scratch;

/* Zero-skipping evaluation (mode 1) of the weak form on Cartesian cells: the
 * same sums as the full evaluation, with the terms whose basis value or
 * derivative is structurally zero left out (the full sums for every mesh are
 * in eval_cell_general). */
static void eval_cell(const or_geom *g, const or_field *f,
                      const double *u, int64_t c, double *out, or_scratch *s) {
  const int d = g->d, k = g->k;
  const int64_t nd = g->nd;
  int cm[OR_MAXD], im[OR_MAXD], qm[OR_MAXD], pm[OR_MAXD];
  cell_multi(g, c, cm);
  const double *uc = u + c * nd;

  for (int64_t q = 0; q < nd; ++q) {
    node_multi(g, q, qm);
    for (int j = 0; j < d; ++j) s->acell[q * d + j] = field_at(g, f, cm, qm, j);
  }

  /* Step 2 of Algorithm 2, interpolation: u_h(x_q) = sum_i' u_i' phi_i'(x_q). */
  for (int64_t q = 0; q < nd; ++q) {
    node_multi(g, q, qm);
    /* Only phi_q is nonzero at x_q (nodal basis, collocated points). */
    s->uh[q] = uc[q] * phi_at(g, qm, qm);
  }

  /* Volume term V_i = sum_q W_q grad phi_i(x_q) . a(x_q) u_h(x_q). */
  for (int64_t i = 0; i < nd; ++i) {
    node_multi(g, i, im);
    double v = 0.0;
    /* d/dx_j phi_i vanishes at x_q unless q agrees with i off dim j. */
    for (int j = 0; j < d; ++j)
      for (int r = 0; r <= k; ++r) {
        for (int m = 0; m < d; ++m) qm[m] = im[m];
        qm[j] = r;
        int64_t q = node_linear(g, qm);
        v += vol_weight(g, qm) * dphi_at(g, im, qm, j) * s->acell[q * d + j] * s->uh[q];
      }
    s->rhs[i] = v;
  }

  /* Face term F_i = sum_faces sum_p W^f_p phi_i(x_p) (a.n) u*(x_p), upwind:
   * u* is the own trace where a.n >= 0 (outflow), else the neighbour's. */
  for (int j = 0; j < d; ++j)
    for (int side = 0; side < 2; ++side) {
      const int pj = side ? k : 0;        /* own node index on this face */
      const int oj = side ? 0 : k;        /* neighbour's node index there */
      const double nj = side ? 1.0 : -1.0; /* outward normal component */
      const int64_t cn = neighbour_cell(g, cm, j, side ? +1 : -1);
      const double *un = u + cn * nd;
      for (int64_t p = 0; p < nd; ++p) {
        node_multi(g, p, pm);
        if (pm[j] != pj) continue; /* face points: nodes with q_j on the face */
        /* Own trace: only phi_p is nonzero at x_p. Neighbour trace: x_p
         * lies on the neighbour's opposite face (node index oj along j), where
         * only the neighbour's basis function of that node is nonzero. */
        for (int m = 0; m < d; ++m) im[m] = pm[m];
        const double uown = uc[p] * phi_at(g, pm, pm);
        im[j] = oj;
        double ph = 1.0;
        for (int m = 0; m < d; ++m) ph *= (m == j) ? g->L[oj][oj] : g->L[pm[m]][pm[m]];
        const double unbr = un[node_linear(g, im)] * ph;
        const double an = s->acell[p * d + j] * nj;
        const double ustar = (an >= 0.0) ? uown : unbr;
        const double Wf = face_weight(g, pm, j);
        /* Only phi_p is nonzero at the node x_p. */
        s->rhs[p] -= Wf * phi_at(g, pm, pm) * an * ustar;
      }
    }

  /* Step 4, inverse mass: the diagonal prod_j h_j M1[i_j]. */
  for (int64_t i = 0; i < nd; ++i) {
    node_multi(g, i, im);
    double m = 1.0;
    for (int j = 0; j < d; ++j) m *= g->h[j] * g->M1[im[j]];
    out[i] = s->rhs[i] / m;
  }
}

/* ------------------------------------------------------------------------ */
/* The same operator with Gauss-Legendre quadrature (mode 2; Sec. 2.5)       */
/* ------------------------------------------------------------------------ */

/* Field component j at the Gauss point qm of cell cm (qm indexes Gauss
 * points; for a face point the normal index is ignored by the field, which
 * does not depend on the coordinate along its own component). a_{x_j} is the
 * velocity coordinate at the Gauss point; a_{v_j} is sign times the nodal
 * interpolant of the E table in the x-cell, evaluated at the x-point. */
static double field_at_gauss(const or_geom *g, const or_field *f, const int *cm,
                             const int *qm, int j) {
  if (f->kind == 0) return f->a[j];
  if (j < g->dx) {
    const int vj = g->dx + j;
    return g->lo[vj] + (cm[vj] + g->gq[qm[vj]]) * g->h[vj];
  }
  int64_t xcell = 0, xs = 1, nxn = 1;
  for (int m = 0; m < g->dx; ++m) {
    xcell += cm[m] * xs;
    xs *= g->cells[m];
    nxn *= g->n;
  }
  double e = 0.0;
  int xm[OR_MAXD];
  for (int64_t xn = 0; xn < nxn; ++xn) {
    int64_t r = xn;
    double ph = 1.0;
    for (int m = 0; m < g->dx; ++m) {
      xm[m] = (int)(r % g->n);
      r /= g->n;
      ph *= g->LG[xm[m]][qm[m]];
    }
    e += f->E[((xcell * nxn) + xn) * g->dx + (j - g->dx)] * ph;
  }
  return f->sign * e;
}

/* phi_i at the Gauss point qm: prod_m l_{i_m}(g_{q_m}). */
static double phi_gauss(const or_geom *g, const int *im, const int *qm) {
  double v = 1.0;
  for (int m = 0; m < g->d; ++m) v *= g->LG[im[m]][qm[m]];
  return v;
}

/* The weak form of Sec. 1.3 with every integral taken by the tensor
 * Gauss-Legendre rule of k+1 points per dimension: volume points g_q, face
 * points the Gauss points in the d-1 tangential dimensions, and the mass
 * matrix this rule integrates exactly, the Kronecker product of h_j MG. */
static void eval_cell_gauss(const or_geom *g, const or_field *f, const double *u,
                            int64_t c, double *out, or_scratch *s) {
  const int d = g->d, k = g->k;
  const int64_t nd = g->nd;
  int cm[OR_MAXD], im[OR_MAXD], qm[OR_MAXD];
  cell_multi(g, c, cm);
  const double *uc = u + c * nd;
  for (int64_t q = 0; q < nd; ++q) node_multi(g, q, s->multi + q * d);

  /* u_h and a at the cell's Gauss points */
  for (int64_t q = 0; q < nd; ++q) {
    memcpy(qm, s->multi + q * d, sizeof(int) * d);
    double v = 0.0;
    for (int64_t ip = 0; ip < nd; ++ip) {
      memcpy(im, s->multi + ip * d, sizeof(int) * d);
      v += uc[ip] * phi_gauss(g, im, qm);
    }
    s->uh[q] = v;
    for (int j = 0; j < d; ++j) s->acell[q * d + j] = field_at_gauss(g, f, cm, qm, j);
  }

  /* V_i = sum_q W_q grad phi_i(g_q) . a(g_q) u_h(g_q), W_q = prod h_m wg_{q_m};
   * d/dx_j phi_i = l'_{i_j} / h_j times the product of the other factors,
   * taken as prefix times suffix product. */
  for (int64_t i = 0; i < nd; ++i) {
    memcpy(im, s->multi + i * d, sizeof(int) * d);
    double v = 0.0;
    for (int64_t q = 0; q < nd; ++q) {
      memcpy(qm, s->multi + q * d, sizeof(int) * d);
      double W = 1.0;
      for (int m = 0; m < d; ++m) W *= g->h[m] * g->wg[qm[m]];
      double pre[OR_MAXD + 1], suf[OR_MAXD + 1];
      pre[0] = 1.0;
      for (int m = 0; m < d; ++m) pre[m + 1] = pre[m] * g->LG[im[m]][qm[m]];
      suf[d] = 1.0;
      for (int m = d - 1; m >= 0; --m) suf[m] = suf[m + 1] * g->LG[im[m]][qm[m]];
      double div = 0.0;
      for (int j = 0; j < d; ++j)
        div += g->DLG[im[j]][qm[j]] / g->h[j] * pre[j] * suf[j + 1] * s->acell[q * d + j];
      v += W * div * s->uh[q];
    }
    s->rhs[i] = v;
  }

  /* F_i = sum over faces and face Gauss points p of W^f_p phi_i(p) (a.n) u*,
   * upwind u*. On the face xi_j = 0 (side 0) or 1 (side 1) only the nodes
   * with i_j on that face have nonzero phi (nodal basis). */
  for (int j = 0; j < d; ++j)
    for (int side = 0; side < 2; ++side) {
      const int pj = side ? k : 0;
      const int oj = side ? 0 : k;
      const double nj = side ? 1.0 : -1.0;
      const int64_t cn = neighbour_cell(g, cm, j, side ? +1 : -1);
      const double *un = u + cn * nd;
      for (int64_t p = 0; p < nd; ++p) {
        memcpy(qm, s->multi + p * d, sizeof(int) * d);
        if (qm[j] != 0) continue; /* one pass over the tangential Gauss points */
        double uown = 0.0, unbr = 0.0;
        for (int64_t ip = 0; ip < nd; ++ip) {
          memcpy(im, s->multi + ip * d, sizeof(int) * d);
          if (im[j] != pj && im[j] != oj) continue; /* zero on both faces */
          double ph = 1.0;
          for (int m = 0; m < d; ++m)
            if (m != j) ph *= g->LG[im[m]][qm[m]];
          if (im[j] == pj) uown += uc[ip] * ph;
          if (im[j] == oj) unbr += un[ip] * ph;
        }
        const double an = field_at_gauss(g, f, cm, qm, j) * nj;
        const double ustar = (an >= 0.0) ? uown : unbr;
        double Wf = 1.0;
        for (int m = 0; m < d; ++m)
          if (m != j) Wf *= g->h[m] * g->wg[qm[m]];
        for (int64_t i = 0; i < nd; ++i) {
          memcpy(im, s->multi + i * d, sizeof(int) * d);
          if (im[j] != pj) continue;
          double ph = 1.0;
          for (int m = 0; m < d; ++m)
            if (m != j) ph *= g->LG[im[m]][qm[m]];
          s->rhs[i] -= Wf * ph * an * ustar;
        }
      }
    }

  /* Inverse mass: the inverse of a Kronecker product is the Kronecker
   * product of the inverses, applied one dimension at a time. */
  for (int64_t i = 0; i < nd; ++i) out[i] = s->rhs[i];
  double line[OR_MAXN];
  for (int j = 0; j < d; ++j)
    for (int64_t b = 0; b < nd; ++b) {
      memcpy(im, s->multi + b * d, sizeof(int) * d);
      if (im[j] != 0) continue;
      for (int r = 0; r <= k; ++r) line[r] = out[b + r * g->nstride[j]];
      for (int r = 0; r <= k; ++r) {
        double v = 0.0;
        for (int q = 0; q <= k; ++q) v += g->MGinv[r][q] * line[q];
        out[b + r * g->nstride[j]] = v / g->h[j];
      }
    }
}

/* ------------------------------------------------------------------------ */
/* The weak form with the metric terms (mapped cells; Sec. 2.5, 3.3)          */
/* ------------------------------------------------------------------------ */

/* Reference point xi (d coordinates in [0,1]) of cell cm: the box point X,
 * the physical point x, |J| and the contravariant field |J| J^{-1} a, with
 * J = d x / d xi block diagonal (the mapped x-block times h, diag(h) for v). */
static void metric_at(const or_geom *g, const or_field *f, const int *cm, const double *xi,
                      const int *qm, int gauss, double *detJ, double *ahat) {
  const int d = g->d, dx = g->dx;
  double X[OR_MAXD], x[OR_MAXD], Jx[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int m = 0; m < d; ++m) X[m] = g->lo[m] + (cm[m] + xi[m]) * g->h[m];
  map_point(g, X, x, Jx);
  /* x-block of J: Jx diag(h_x); its determinant and |J_x| J_x^{-1} by
   * cofactors (adjugate). */
  double A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int m = 0; m < dx; ++m)
    for (int kk = 0; kk < dx; ++kk) A[m][kk] = Jx[m][kk] * g->h[kk];
  double detx, adj[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  if (dx == 1) {
    detx = A[0][0];
    adj[0][0] = 1.0;
  } else if (dx == 2) {
    detx = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    adj[0][0] = A[1][1];
    adj[0][1] = -A[0][1];
    adj[1][0] = -A[1][0];
    adj[1][1] = A[0][0];
  } else {
    detx = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        /* adj[r][cc] = cofactor of A[cc][r] */
        const int r1 = (cc + 1) % 3, r2 = (cc + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        adj[r][cc] = A[r1][c1] * A[r2][c2] - A[r1][c2] * A[r2][c1];
      }
  }
  double detv = 1.0;
  for (int m = dx; m < d; ++m) detv *= g->h[m];
  *detJ = detx * detv;
  /* physical field at the point */
  double a[OR_MAXD];
  for (int j = 0; j < d; ++j)
    a[j] = gauss ? field_at_gauss(g, f, cm, qm, j) : field_at(g, f, cm, qm, j);
  /* |J| J^{-1} a: x-block detv * adj(A) a_x, v-block detx * detv / h a_v */
  for (int j = 0; j < dx; ++j) {
    double s = 0.0;
    for (int kk = 0; kk < dx; ++kk) s += adj[j][kk] * a[kk];
    ahat[j] = detv * s;
  }
  for (int j = dx; j < d; ++j) ahat[j] = detx * detv / g->h[j] * a[j];
}

/* The weak form of Sec. 1.3 on a mapped cell with quadrature at the GL
 * points (gauss = 0: nodal, diagonal mass W |J|) or the Gauss points
 * (gauss = 1: mass B^T diag(W |J|) B per cell, B[q][i] = l_i(g_q) square,
 * inverted as B^{-1} diag(W |J|)^{-1} B^{-T}):
 *   V_i = sum_q W_q sum_j d/dxi_j phi_i(q) ahat_j(q) u_h(q),
 *   F_i = sum_faces sum_p W^f_p phi_i(p) (ahat_j n_j)(p) u*(p), upwind u*,
 * with reference weights W and the reference normal n_j = -1 / +1. */
static void eval_cell_general(const or_geom *g, const or_field *f, int gauss,
                              const double *u, int64_t c, double *out, or_scratch *s) {
  const int d = g->d, k = g->k;
  const int64_t nd = g->nd;
  const double *pt = gauss ? g->gq : g->xi;
  const double *wt = gauss ? g->wg : g->w;
  int cm[OR_MAXD], im[OR_MAXD], qm[OR_MAXD];
  cell_multi(g, c, cm);
  const double *uc = u + c * nd;
  for (int64_t q = 0; q < nd; ++q) node_multi(g, q, s->multi + q * d);
  /* L1[m][q] = l_m(pt_q), D1[m][q] = l_m'(pt_q) */
  double L1[OR_MAXN][OR_MAXN], D1[OR_MAXN][OR_MAXN];
  for (int m = 0; m <= k; ++m)
    for (int q = 0; q <= k; ++q) {
      L1[m][q] = gauss ? g->LG[m][q] : g->L[m][q];
      D1[m][q] = gauss ? g->DLG[m][q] : g->DL[m][q];
    }
  /* u_h, |J| and ahat at the cell's quadrature points; acell holds ahat,
   * rhs temporarily nothing */
  double *detJ = (double *)malloc(sizeof(double) * nd);
  for (int64_t q = 0; q < nd; ++q) {
    memcpy(qm, s->multi + q * d, sizeof(int) * d);
    double xi[OR_MAXD];
    for (int m = 0; m < d; ++m) xi[m] = pt[qm[m]];
    metric_at(g, f, cm, xi, qm, gauss, &detJ[q], s->acell + q * d);
    double v = 0.0;
    for (int64_t ip = 0; ip < nd; ++ip) {
      memcpy(im, s->multi + ip * d, sizeof(int) * d);
      double ph = 1.0;
      for (int m = 0; m < d; ++m) ph *= L1[im[m]][qm[m]];
      v += uc[ip] * ph;
    }
    s->uh[q] = v;
  }
  for (int64_t i = 0; i < nd; ++i) {
    memcpy(im, s->multi + i * d, sizeof(int) * d);
    double v = 0.0;
    for (int64_t q = 0; q < nd; ++q) {
      memcpy(qm, s->multi + q * d, sizeof(int) * d);
      double W = 1.0;
      for (int m = 0; m < d; ++m) W *= wt[qm[m]];
      for (int j = 0; j < d; ++j) {
        double dphi = D1[im[j]][qm[j]];
        for (int m = 0; m < d; ++m)
          if (m != j) dphi *= L1[im[m]][qm[m]];
        v += W * dphi * s->acell[q * d + j] * s->uh[q];
      }
    }
    s->rhs[i] = v;
  }
  for (int j = 0; j < d; ++j)
    for (int side = 0; side < 2; ++side) {
      const int pj = side ? k : 0, oj = side ? 0 : k;
      const double nj = side ? 1.0 : -1.0;
      const int64_t cn = neighbour_cell(g, cm, j, side ? +1 : -1);
      const double *un = u + cn * nd;
      for (int64_t p = 0; p < nd; ++p) {
        memcpy(qm, s->multi + p * d, sizeof(int) * d);
        if (qm[j] != 0) continue; /* one pass over the tangential points */
        double xi[OR_MAXD];
        for (int m = 0; m < d; ++m) xi[m] = pt[qm[m]];
        xi[j] = side ? 1.0 : 0.0;
        double dJ, ah[OR_MAXD];
        metric_at(g, f, cm, xi, qm, gauss, &dJ, ah);
        double uown = 0.0, unbr = 0.0;
        for (int64_t ip = 0; ip < nd; ++ip) {
          memcpy(im, s->multi + ip * d, sizeof(int) * d);
          if (im[j] != pj && im[j] != oj) continue;
          double ph = 1.0;
          for (int m = 0; m < d; ++m)
            if (m != j) ph *= L1[im[m]][qm[m]];
          if (im[j] == pj) uown += uc[ip] * ph;
          if (im[j] == oj) unbr += un[ip] * ph;
        }
        const double an = ah[j] * nj;
        const double ustar = an >= 0.0 ? uown : unbr;
        double Wf = 1.0;
        for (int m = 0; m < d; ++m)
          if (m != j) Wf *= wt[qm[m]];
        for (int64_t i = 0; i < nd; ++i) {
          memcpy(im, s->multi + i * d, sizeof(int) * d);
          if (im[j] != pj) continue;
          double ph = 1.0;
          for (int m = 0; m < d; ++m)
            if (m != j) ph *= L1[im[m]][qm[m]];
          s->rhs[i] -= Wf * ph * an * ustar;
        }
      }
    }
  /* inverse mass */
  for (int64_t i = 0; i < nd; ++i) out[i] = s->rhs[i];
  double line[OR_MAXN];
  if (gauss) {
    /* out <- (B^{-T})^{x d} out: per dimension y = B^{-T} r */
    for (int j = 0; j < d; ++j)
      for (int64_t b = 0; b < nd; ++b) {
        memcpy(im, s->multi + b * d, sizeof(int) * d);
        if (im[j] != 0) continue;
        for (int r = 0; r <= k; ++r) line[r] = out[b + r * g->nstride[j]];
        for (int q = 0; q <= k; ++q) {
          double v = 0.0;
          for (int r = 0; r <= k; ++r) v += g->Binv[r][q] * line[r];
          out[b + q * g->nstride[j]] = v;
        }
      }
  }
  for (int64_t q = 0; q < nd; ++q) {
    memcpy(qm, s->multi + q * d, sizeof(int) * d);
    double W = 1.0;
    for (int m = 0; m < d; ++m) W *= wt[qm[m]];
    out[q] /= W * detJ[q];
  }
  if (gauss) {
    /* out <- (B^{-1})^{x d} out */
    for (int j = 0; j < d; ++j)
      for (int64_t b = 0; b < nd; ++b) {
        memcpy(im, s->multi + b * d, sizeof(int) * d);
        if (im[j] != 0) continue;
        for (int r = 0; r <= k; ++r) line[r] = out[b + r * g->nstride[j]];
        for (int q = 0; q <= k; ++q) {
          double v = 0.0;
          for (int r = 0; r <= k; ++r) v += g->Binv[q][r] * line[r];
          out[b + q * g->nstride[j]] = v;
        }
      }
  }
  free(detJ);
}

int or_apply_cells(const or_mesh *mesh, int k, const or_field *field, int mode,
                   const double *u, const int64_t *cells, int64_t ncells,
                   double *out) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || check_field(&g, field)) return -1;
  if (mode < 0 || mode > 3 || (mode == 1 && g.eps != 0.0)) return -1;
  for (int64_t t = 0; t < ncells; ++t)
    if (cells[t] < 0 || cells[t] >= g.ncells) return -1;
  int err = 0;
#pragma omp parallel
  {
    or_scratch s;
    s.uh = (double *)malloc(sizeof(double) * g.nd);
    s.rhs = (double *)malloc(sizeof(double) * g.nd);
    s.acell = (double *)malloc(sizeof(double) * g.nd * g.d);
    s.multi = (int *)malloc(sizeof(int) * g.nd * g.d);
    if (!s.uh || !s.rhs || !s.acell || !s.multi) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(dynamic, 4)
      for (int64_t t = 0; t < ncells; ++t) {
        if (mode == 0)
          eval_cell_general(&g, field, 0, u, cells[t], out + t * g.nd, &s);
        else if (mode == 3 || (mode == 2 && g.eps != 0.0))
          eval_cell_general(&g, field, 1, u, cells[t], out + t * g.nd, &s);
        else if (mode == 2)
          eval_cell_gauss(&g, field, u, cells[t], out + t * g.nd, &s);
        else
          eval_cell(&g, field, u, cells[t], out + t * g.nd, &s);
      }
    }
    free(s.uh);
    free(s.rhs);
    free(s.acell);
    free(s.multi);
  }
  return err ? -1 : 0;
}

int or_apply(const or_mesh *mesh, int k, const or_field *field, int mode,
             const double *u, double *out) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
  int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * g.ncells);
  if (!cells) return -1;
  for (int64_t c = 0; c < g.ncells; ++c) cells[c] = c;
  int r = or_apply_cells(mesh, k, field, mode, u, cells, g.ncells, out);
  free(cells);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Low-storage Runge-Kutta (Sec. 5.4: order 4, 5 stages, 3 vectors)         */
/* ------------------------------------------------------------------------ */

/* Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage scheme:
 * per stage  du <- A_s du + dt L(u),  u <- u + B_s du. */
void or_lsrk45_coefficients(double *A, double *B, double *C) {
  A[0] = 0.0;
  A[1] = -567301805773.0 / 1357537059087.0;
  A[2] = -2404267990393.0 / 2016746695238.0;
  A[3] = -3550918686646.0 / 2091501179385.0;
  A[4] = -1275806237668.0 / 842570457699.0;
  B[0] = 1432997174477.0 / 9575080441755.0;
  B[1] = 5161836677717.0 / 13612068292357.0;
  B[2] = 1720146321549.0 / 2090206949498.0;
  B[3] = 3134564353537.0 / 4481467310338.0;
  B[4] = 2277821191437.0 / 14882151754819.0;
  C[0] = 0.0;
  C[1] = 1432997174477.0 / 9575080441755.0;
  C[2] = 2526269341429.0 / 6820363962896.0;
  C[3] = 2006345519317.0 / 3224310063776.0;
  C[4] = 2802321613138.0 / 2924317926251.0;
}

int or_rk_stage(const or_mesh *mesh, int k, const or_field *field, int mode, double dt,
                int stage, double *u, double *du, double *L) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || check_field(&g, field)) return -1;
  if (stage < 0 || stage > 4) return -1;
  const int64_t N = g.nd * g.ncells;
  double A[5], B[5], C[5];
  or_lsrk45_coefficients(A, B, C);
  const int r = or_apply(mesh, k, field, mode, u, L);
  if (r) return r;
  /* A_1 = 0: the first stage does not read du (which may hold anything). */
  const double a = A[stage], b = B[stage];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    du[i] = (stage == 0 ? 0.0 : a * du[i]) + dt * L[i];
    u[i] = u[i] + b * du[i];
  }
  return 0;
}

int or_rk_steps(const or_mesh *mesh, int k, const or_field *field, int mode,
                double dt, int nsteps, double *u) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || check_field(&g, field)) return -1;
  const int64_t N = g.nd * g.ncells;
  double *du = (double *)calloc((size_t)N, sizeof(double));
  double *L = (double *)malloc(sizeof(double) * (size_t)N);
  if (!du || !L) {
    free(du);
    free(L);
    return -1;
  }
  int r = 0;
  for (int step = 0; step < nsteps && !r; ++step)
    for (int st = 0; st < 5 && !r; ++st) r = or_rk_stage(mesh, k, field, mode, dt, st, u, du, L);
  free(du);
  free(L);
  return r;
}

double or_stable_dt(const or_mesh *mesh, int k, const or_field *field,
                    double cfl) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || check_field(&g, field)) return -1.0;
  double sum = 0.0;
  for (int j = 0; j < g.d; ++j) {
    double amax = 0.0;
    if (field->kind == 0) {
      amax = fabs(field->a[j]);
    } else if (j < g.dx) {
      /* |v_j| is largest at a node of the velocity mesh. */
      const int vj = g.dx + j;
      for (int c = 0; c < g.cells[vj]; ++c)
        for (int q = 0; q <= k; ++q) {
          double v = g.lo[vj] + (c + g.xi[q]) * g.h[vj];
          if (fabs(v) > amax) amax = fabs(v);
        }
    } else {
      int64_t nx = 1;
      for (int m = 0; m < g.dx; ++m) nx *= (int64_t)g.cells[m];
      for (int m = 0; m < g.dx; ++m) nx *= g.n;
      for (int64_t t = 0; t < nx; ++t) {
        double v = fabs(field->sign * field->E[t * g.dx + (j - g.dx)]);
        if (v > amax) amax = v;
      }
    }
    sum += amax / g.h[j];
  }
  if (!(sum > 0.0)) return -1.0;
  return cfl / ((2.0 * k + 1.0) * sum);
}

int or_init_state(const or_mesh *mesh, int k, int kind, const double *params,
                  double *u) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
  if (kind != 0 && kind != 1) return -1;
  const double alpha = (kind == 1 && params) ? params[0] : 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < g.ncells; ++c) {
    int cm[OR_MAXD], qm[OR_MAXD];
    cell_multi(&g, c, cm);
    for (int64_t q = 0; q < g.nd; ++q) {
      node_multi(&g, q, qm);
      double v;
      if (kind == 0) {
        v = 1.0;
        for (int j = 0; j < g.d; ++j) {
          double x = node_coord(&g, cm, qm, j);
          v *= sin(2.0 * OR_PI * (x - g.lo[j]) / (g.hi[j] - g.lo[j]));
        }
      } else {
        double x1 = node_coord(&g, cm, qm, 0);
        double v2 = 0.0;
        for (int j = g.dx; j < g.d; ++j) {
          double vj = node_coord(&g, cm, qm, j);
          v2 += vj * vj;
        }
        v = (1.0 + alpha * cos(2.0 * OR_PI * (x1 - g.lo[0]) / (g.hi[0] - g.lo[0]))) *
            pow(2.0 * OR_PI, -0.5 * g.dv) * exp(-0.5 * v2);
      }
      u[c * g.nd + q] = v;
    }
  }
  return 0;
}

int or_field_sine_table(const or_mesh *mesh, int k, double amp, double *E) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
  int64_t nxc = 1, nxn = 1;
  for (int m = 0; m < g.dx; ++m) {
    nxc *= g.cells[m];
    nxn *= g.n;
  }
  for (int64_t xc = 0; xc < nxc; ++xc)
    for (int64_t xn = 0; xn < nxn; ++xn) {
      int64_t cr = xc, nr = xn;
      for (int m = 0; m < g.dx; ++m) {
        int cmm = (int)(cr % g.cells[m]);
        int qmm = (int)(nr % g.n);
        cr /= g.cells[m];
        nr /= g.n;
        (void)cmm;
        (void)qmm;
        int cfull[OR_MAXD] = {0}, qfull[OR_MAXD] = {0};
        {
          int64_t cr2 = xc, nr2 = xn;
          for (int mm = 0; mm < g.dx; ++mm) {
            cfull[mm] = (int)(cr2 % g.cells[mm]);
            qfull[mm] = (int)(nr2 % g.n);
            cr2 /= g.cells[mm];
            nr2 /= g.n;
          }
        }
        double x = node_coord(&g, cfull, qfull, m);
        E[(xc * nxn + xn) * g.dx + m] =
            amp * sin(2.0 * OR_PI * (x - g.lo[m]) / (g.hi[m] - g.lo[m]));
      }
    }
  return 0;
}

int or_diagnostics(const or_mesh *mesh, int k, const double *u, double *mass,
                   double *energy) {
  or_geom g;
  if (setup_geom(mesh, k, &g)) return -1;
  double ms = 0.0, en = 0.0;
#pragma omp parallel for reduction(+ : ms, en) schedule(static)
  for (int64_t c = 0; c < g.ncells; ++c) {
    int qm[OR_MAXD], cm[OR_MAXD];
    cell_multi(&g, c, cm);
    for (int64_t q = 0; q < g.nd; ++q) {
      node_multi(&g, q, qm);
      double W = vol_weight(&g, qm);
      if (g.eps != 0.0) {
        /* times det(dx/dX) of the mapping at the node */
        double X[OR_MAXD], x[OR_MAXD], Jx[3][3];
        for (int m = 0; m < g.d; ++m) X[m] = g.lo[m] + (cm[m] + g.xi[qm[m]]) * g.h[m];
        map_point(&g, X, x, Jx);
        double dt = Jx[0][0];
        if (g.dx == 2) dt = Jx[0][0] * Jx[1][1] - Jx[0][1] * Jx[1][0];
        if (g.dx == 3)
          dt = Jx[0][0] * (Jx[1][1] * Jx[2][2] - Jx[1][2] * Jx[2][1]) -
               Jx[0][1] * (Jx[1][0] * Jx[2][2] - Jx[1][2] * Jx[2][0]) +
               Jx[0][2] * (Jx[1][0] * Jx[2][1] - Jx[1][1] * Jx[2][0]);
        W *= dt;
      }
      double v = u[c * g.nd + q];
      ms += W * v;
      en += W * v * v;
    }
  }
  *mass = ms;
  *energy = en;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Vlasov-Poisson field (Sec. 6)                                            */
/* ------------------------------------------------------------------------ */

/* The x-points are the x-nodes of the x-cells: p = xcell * n^dx + xnode, both
 * lexicographic with dim 1 fastest - the layout of the E table. */
static void x_layout(const or_geom *g, int64_t *nxc, int64_t *nxn, int64_t *nvc,
                     int64_t *nvn) {
  *nxc = *nxn = *nvc = *nvn = 1;
  for (int j = 0; j < g->dx; ++j) {
    *nxc *= g->cells[j];
    *nxn *= g->n;
  }
  for (int j = g->dx; j < g->d; ++j) {
    *nvc *= g->cells[j];
    *nvn *= g->n;
  }
}

/* Coordinates and quadrature weight prod_j h_j w_{i_j} of x-point p. */
static double x_point(const or_geom *g, int64_t p, int64_t nxn, double *x) {
  int64_t xc = p / nxn, xn = p % nxn;
  double W = 1.0;
  for (int j = 0; j < g->dx; ++j) {
    const int c = (int)(xc % g->cells[j]), i = (int)(xn % g->n);
    xc /= g->cells[j];
    xn /= g->n;
    x[j] = g->lo[j] + (c + g->xi[i]) * g->h[j];
    W *= g->h[j] * g->w[i];
  }
  return W;
}

int or_vp_density(const or_mesh *mesh, int k, const double *u, double *rho) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || g.eps != 0.0 || g.dx != g.dv) return -1;
  int64_t nxc, nxn, nvc, nvn;
  x_layout(&g, &nxc, &nxn, &nvc, &nvn);
  const int64_t X = nxc * nxn;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < X; ++p) {
    const int64_t xc = p / nxn, xn = p % nxn;
    double s = 0.0;
    for (int64_t cv = 0; cv < nvc; ++cv)
      for (int64_t vn = 0; vn < nvn; ++vn) {
        /* velocity quadrature weight prod_j h_{v_j} w_{i_{v_j}} */
        double Wv = 1.0;
        int64_t r = vn;
        for (int j = g.dx; j < g.d; ++j) {
          Wv *= g.h[j] * g.w[r % g.n];
          r /= g.n;
        }
        const int64_t cell = xc + nxc * cv, node = xn + nxn * vn;
        s += Wv * u[cell * g.nd + node];
      }
    rho[p] = s;
  }
  return 0;
}

int or_vp_field(const or_mesh *mesh, int k, int M, const double *rho, double *E) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || g.eps != 0.0 || g.dx != g.dv || M < 1) return -1;
  int64_t nxc, nxn, nvc, nvn;
  x_layout(&g, &nxc, &nxn, &nvc, &nvn);
  const int64_t X = nxc * nxn;
  double vol = 1.0;
  for (int j = 0; j < g.dx; ++j) vol *= g.hi[j] - g.lo[j];
  for (int64_t i = 0; i < X * g.dx; ++i) E[i] = 0.0;
  int64_t nmodes = 1;
  for (int j = 0; j < g.dx; ++j) nmodes *= 2 * M + 1;
  for (int64_t mi = 0; mi < nmodes; ++mi) {
    /* wave vector k_j = 2 pi m_j / L_j, m_j in -M..M */
    double kv[3] = {0, 0, 0}, k2 = 0.0;
    int64_t r = mi;
    int zero = 1;
    for (int j = 0; j < g.dx; ++j) {
      const int m = (int)(r % (2 * M + 1)) - M;
      r /= 2 * M + 1;
      if (m) zero = 0;
      kv[j] = 2.0 * OR_PI * m / (g.hi[j] - g.lo[j]);
      k2 += kv[j] * kv[j];
    }
    if (zero) continue; /* the mean is balanced by the background */
    /* rho_hat = (1/|Omega_x|) int rho exp(-i k.x) dx, GL quadrature in x */
    double re = 0.0, im = 0.0;
    for (int64_t p = 0; p < X; ++p) {
      double x[3];
      const double W = x_point(&g, p, nxn, x);
      double ph = 0.0;
      for (int j = 0; j < g.dx; ++j) ph += kv[j] * x[j];
      re += W * rho[p] * cos(ph);
      im -= W * rho[p] * sin(ph);
    }
    re /= vol;
    im /= vol;
    /* -Laplace phi = 1 - rho, E = -grad phi: E_hat_j = i k_j rho_hat / |k|^2 */
    for (int64_t p = 0; p < X; ++p) {
      double x[3];
      x_point(&g, p, nxn, x);
      double ph = 0.0;
      for (int j = 0; j < g.dx; ++j) ph += kv[j] * x[j];
      const double c = cos(ph), s = sin(ph);
      for (int j = 0; j < g.dx; ++j) {
        const double cre = -kv[j] / k2 * im, cim = kv[j] / k2 * re;
        E[p * g.dx + j] += cre * c - cim * s; /* Re[(cre + i cim) exp(i ph)] */
      }
    }
  }
  return 0;
}

int or_vp_rk_steps(const or_mesh *mesh, int k, int M, int mode, double dt, int nsteps,
                   double *u) {
  or_geom g;
  if (setup_geom(mesh, k, &g) || g.eps != 0.0 || g.dx != g.dv) return -1;
  int64_t nxc, nxn, nvc, nvn;
  x_layout(&g, &nxc, &nxn, &nvc, &nvn);
  const int64_t X = nxc * nxn, N = g.nd * g.ncells;
  double A[5], B[5], C[5];
  or_lsrk45_coefficients(A, B, C);
  double *du = (double *)calloc((size_t)N, sizeof(double));
  double *L = (double *)malloc(sizeof(double) * (size_t)N);
  double *rho = (double *)malloc(sizeof(double) * (size_t)X);
  double *E = (double *)malloc(sizeof(double) * (size_t)(X * g.dx));
  int r = (!du || !L || !rho || !E) ? -1 : 0;
  or_field f;
  memset(&f, 0, sizeof(f));
  f.kind = 1;
  f.E = E;
  f.sign = -1.0; /* electrons: a = (v, -E) */
  for (int step = 0; step < nsteps && !r; ++step)
    for (int st = 0; st < 5 && !r; ++st) {
      /* the field of the stage's own input */
      r = or_vp_density(mesh, k, u, rho);
      if (!r) r = or_vp_field(mesh, k, M, rho, E);
      if (!r) r = or_apply(mesh, k, &f, mode, u, L);
      if (r) break;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        du[i] = A[st] * du[i] + dt * L[i];
        u[i] = u[i] + B[st] * du[i];
      }
    }
  free(du);
  free(L);
  free(rho);
  free(E);
  return r;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
