/*
 * Plain CPU oracle for the upwind, Gauss-Lobatto-collocation DG advection
 * operator on a periodic Cartesian box and its low-storage RK integrator.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes
 * or calls this code; it exists so that tests and the benchmark's CPU
 * baseline can check the GPU path against a slow, obviously correct
 * evaluation of the same discrete operator. It shares no source with the
 * GPU library.
 *
 * Paper: Munch, Kormann, Kronbichler, "hyper.deal: An efficient, matrix-free
 * finite-element library for high-dimensional partial differential
 * equations" (arXiv 2002.08110).
 *
 *  - Model problem: conservative advection df/dt + div(a f) = 0 with periodic
 *    boundaries (Sec. 1.2, eq. intro:advection); for phase space the field is
 *    a = (v, E(x)) (Sec. 1.2, eq. intro:vp:simple; Sec. 6.1).
 *  - DG weak form with a numerical flux (Sec. 1.3), nodal tensor-product
 *    basis on Gauss-Lobatto points (Sec. 2.3), Gauss-Lobatto quadrature in
 *    the same points (collocation, Sec. 2.5), diagonal mass matrix (Sec. 1.3).
 *  - Element-centric evaluation of one cell with its 2d faces (Sec. 3.4,
 *    Algorithms 1 and 2).
 *  - Five-stage, fourth-order low-storage Runge-Kutta scheme with three
 *    solution-sized vectors (Sec. 5.4).
 *
 * Every function is parity-pinned by the CPU tests (tests/test_oracle_*.py)
 * against closed forms, invariants and exact solutions; none is "parity
 * unpinned".
 */
#ifndef HD_ORACLE_H
#define HD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Periodic Cartesian box, dim_x configuration dims first, then dim_v
 * velocity dims; cells[j] cells of width (hi[j]-lo[j])/cells[j] in dim j. */
typedef struct {
  int dim_x, dim_v;
  int cells[6];
  double lo[6], hi[6];
  /* Deformation of the configuration space (the tensor-product mapping of
   * Sec. 3.1/3.3 with a curved x-mesh and a Cartesian v-mesh): the box point
   * X maps to x_m = X_m + map_eps L_m prod_{k < dim_x} sin(2 pi (X_k - lo_k)
   * / L_k), L = hi - lo. 0: Cartesian. |map_eps| <= 0.05. */
  double map_eps;
} or_mesh;

/* Advection field.
 *  kind 0: constant a[0..d-1].
 *  kind 1: phase space, a_{x_j} = v_j (the coordinate of velocity dim j) and
 *          a_{v_j} = sign * E_j(x), with E given at the x-nodes:
 *          E[((xcell * n^dx) + xnode) * dx + j], xcell lexicographic over the
 *          x-cells (dim 1 fastest), xnode lexicographic over the x-node
 *          indices (dim 1 fastest). Requires dim_x == dim_v. */
typedef struct {
  int kind;
  double a[6];
  const double *E;
  double sign;
} or_field;

/* Gauss-Lobatto rule with k+1 points on [0,1]; xi ascending, sum w = 1.
 * Returns 0, or -1 for k < 1 or k > 16. */
int or_gl_rule(int k, double *xi, double *w);

/* Lagrange polynomial l_m on the GL points of degree k, and its derivative. */
double or_lagrange(int k, const double *xi, int m, double x);
double or_lagrange_deriv(int k, const double *xi, int m, double x);

/* Number of DoFs, n^d * prod(cells). */
int64_t or_num_dofs(const or_mesh *mesh, int k);

/* Node coordinates: X[dof * d + j] for the canonical DoF numbering
 * (dof = cell * n^d + node, cell and node lexicographic, dim 1 fastest). */
int or_node_coords(const or_mesh *mesh, int k, double *X);

/* Gauss-Legendre rule with k+1 points on [0,1]; g ascending, sum w = 1. */
int or_gauss_rule(int k, double *g, double *w);

/* Evaluate out = M^{-1} A(u) for the listed cells (out holds n^d values per
 * listed cell, in list order). mode 0: full basis (every phi_i evaluated at
 * every quadrature point); mode 1: the same sums with structurally zero
 * basis values skipped; mode 2: the same weak form with Gauss-Legendre
 * quadrature (k+1 points per dimension, full sums, the exactly integrated
 * non-diagonal mass matrix; the E table enters through its nodal
 * interpolant). Every function taking a mode accepts 2. With a mapping
 * (map_eps != 0) modes 0 and 2 evaluate the weak form with the metric
 * terms (contravariant flux |J| J^{-1} a at the quadrature points, the mass
 * matrix with |J|); mode 1 requires map_eps = 0. Mode 3 is mode 2 through
 * that general evaluation even without a mapping (for tests). Returns 0,
 * or -1 on invalid input. */
int or_apply_cells(const or_mesh *mesh, int k, const or_field *field, int mode,
                   const double *u, const int64_t *cells, int64_t ncells,
                   double *out);

/* out = M^{-1} A(u) on all cells. */
int or_apply(const or_mesh *mesh, int k, const or_field *field, int mode,
             const double *u, double *out);

/* The 2N-storage, five-stage, fourth-order RK coefficients (A, B, C). */
void or_lsrk45_coefficients(double *A, double *B, double *C);

/* Stage `stage` (0..4) of the low-storage RK scheme (Sec. 5.4; the
 * Carpenter-Kennedy 2N coefficients) in place: L = L(u) (scratch of N
 * values), du <- A_s du + dt L (du is not read at stage 0, A_1 = 0),
 * u <- u + B_s du. */
int or_rk_stage(const or_mesh *mesh, int k, const or_field *field, int mode, double dt,
                int stage, double *u, double *du, double *L);

/* nsteps steps of the low-storage RK scheme with time step dt, in place on u
 * (five calls of or_rk_stage per step, du starting at zero). */
int or_rk_steps(const or_mesh *mesh, int k, const or_field *field, int mode,
                double dt, int nsteps, double *u);

/* dt = cfl / ((2k+1) * sum_j max|a_j| / h_j). */
double or_stable_dt(const or_mesh *mesh, int k, const or_field *field,
                    double cfl);

/* Initial state by nodal interpolation.
 *  kind 0: prod_j sin(2 pi (x_j - lo_j)/(hi_j - lo_j)).
 *  kind 1: (1 + p[0] cos(2 pi (x_1 - lo_1)/(hi_1 - lo_1)))
 *          * (2 pi)^(-dv/2) exp(-|v|^2 / 2). */
int or_init_state(const or_mesh *mesh, int k, int kind, const double *params,
                  double *u);

/* E_j(x) = amp * sin(2 pi (x_j - lo_j)/(hi_j - lo_j)) tabulated at x-nodes. */
int or_field_sine_table(const or_mesh *mesh, int k, double amp, double *E);

/* mass = sum W_i u_i, energy = sum W_i u_i^2, W_i = prod_j h_j w_{i_j}. */
int or_diagnostics(const or_mesh *mesh, int k, const double *u, double *mass,
                   double *energy);

/* Vlasov-Poisson field (Sec. 6; electrons on a neutralizing background,
 * dim_x == dim_v), with x-points p = xcell * n^dx + xnode as in the E table:
 *  or_vp_density: rho(x_p) = int f(x_p, v) dv, Gauss-Lobatto quadrature in v
 *                 (exact for the DG polynomial).
 *  or_vp_field:   -Laplace phi = 1 - rho, E = -grad phi on the periodic x-box,
 *                 solved spectrally with the modes m in [-M, M]^dx, m != 0:
 *                 rho_hat_m = |Omega_x|^-1 sum_p W_p rho_p exp(-i k_m.x_p)
 *                 (GL quadrature in x), k_m = 2 pi m / L, and
 *                 E(x_p) = sum_m Re[i k_m rho_hat_m / |k_m|^2 exp(i k_m.x_p)];
 *                 E[p * dx + j] as the or_field table.
 *  or_vp_rk_steps: LSRK steps of f_t + v.grad_x f - E.grad_v f = 0 with the
 *                 field recomputed from each stage's input (a = (v, -E)). */
int or_vp_density(const or_mesh *mesh, int k, const double *u, double *rho);
int or_vp_field(const or_mesh *mesh, int k, int M, const double *rho, double *E);
int or_vp_rk_steps(const or_mesh *mesh, int k, int M, int mode, double dt, int nsteps,
                   double *u);

/* Number of OpenMP threads the oracle uses. */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
