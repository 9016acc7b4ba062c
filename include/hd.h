/*
 * hd.h - C ABI of the MI355X (gfx950) library for the matrix-free,
 * upwind, Gauss-Lobatto-collocation discontinuous Galerkin advection
 * operator in 2 to 6 dimensions on a tensor product of a configuration-space
 * mesh and a velocity-space mesh, advanced by a five-stage fourth-order
 * low-storage Runge-Kutta scheme.
 *
 * Paper: Munch, Kormann, Kronbichler, "hyper.deal: An efficient,
 * matrix-free finite-element library for high-dimensional partial
 * differential equations", arXiv 2002.08110.
 *
 * General conventions (every function):
 *  - Return value: hd_status; HD_OK (0) on success, a negative code on error.
 *    The message of the last error on the calling thread is returned by
 *    hd_last_error(). No C++ exception crosses this boundary.
 *  - Streams: `hd_stream` is a hipStream_t passed as void*; NULL is the
 *    default stream. Work is enqueued asynchronously on that stream unless a
 *    function says it synchronizes.
 *  - Ownership: an hd_solver belongs to the caller from hd_create until
 *    hd_destroy. Device memory handed to hd_bind belongs to the caller and
 *    must outlive the solver's use; the library never frees it. Host arrays
 *    are only read (or written) during the call.
 *  - Canonical DoF layout (the layout of every state vector crossing the
 *    ABI): dof = cell * (k+1)^d + node. The cell index is lexicographic over
 *    (c_1..c_d) with dimension 1 fastest, dimensions ordered x_1..x_dx then
 *    v_1..v_dv (x-fastest cell enumeration, Sec. 3.2); the node index is
 *    lexicographic over the Gauss-Lobatto node indices (i_1..i_d), dimension
 *    1 fastest. Nodes lie at lo_j + (c_j + xi_{i_j}) h_j with xi the
 *    Gauss-Lobatto points on [0,1] (Sec. 2.3).
 *  - Errors: HD_ERR_INVALID for bad arguments (dim_x or dim_v outside 1..3,
 *    degree < 1, a cell count < 1, lo >= hi, NULL pointers, a call that needs
 *    bound memory before hd_bind, a buffer smaller than required);
 *    HD_ERR_UNSUPPORTED for valid input with no compiled kernel (degree > 5);
 *    HD_ERR_HIP when a HIP call fails (its message is kept).
 */
#ifndef HD_H
#define HD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HD_OK = 0,
  HD_ERR_INVALID = -1,
  HD_ERR_UNSUPPORTED = -2,
  HD_ERR_OOM = -3,
  HD_ERR_HIP = -4,
  HD_ERR_STATE = -5
} hd_status;

/* Operator precision. HD_FP64: operator, stage increment and solution in
 * FP64 (the paper's precision throughout). HD_FP32_OP_FP64_ACC: operator and
 * stage increment du in FP32 (FP32 accumulation of the sums); the solution
 * u, its RK accumulation and the diagnostics stay FP64. */
typedef enum { HD_FP64 = 0, HD_FP32_OP_FP64_ACC = 1 } hd_precision;

/* Periodic Cartesian box: the tensor product of a dim_x-dimensional
 * configuration mesh and a dim_v-dimensional velocity mesh (Sec. 3.1),
 * x dims first. cells[j] cells of width (hi[j]-lo[j])/cells[j] in dim j;
 * entries beyond dim_x + dim_v are ignored. */
typedef struct {
  int dim_x, dim_v;
  int cells[6];
  double lo[6], hi[6];
} hd_mesh;

typedef void *hd_stream;             /* hipStream_t */
typedef struct hd_solver hd_solver;  /* opaque */
typedef struct hd_batch hd_batch;    /* opaque */

/* Launch plan of the fused stage kernel (chosen by the autotuner).
 *  lds:        1 = stage each cell's values in LDS for the sweeps along
 *              thread-distributed dimensions; 0 = read them from global memory.
 *  cells_per_wg: units per workgroup (lds = 1): cells, or slabs of cells if
 *              split_dims > 0 - ignored for lds = 0.
 *  wg_size:    threads per workgroup for lds = 0 (multiple of 64, <= 1024).
 *  xcd_remap:  1 = map consecutive cell tiles to the same XCD.
 *  reg_dims:   number of slowest dimensions whose lines a thread keeps in
 *              registers (1 or 2; at most dim_v).
 *  kernel:     0 = the generic kernel (the fields above apply); 2 = the
 *              dimension-split passes for d = 6 (3 x + 3 v) and d = 5 (3 x +
 *              2 v) at degrees 4 and 5 with collocation on Cartesian cells:
 *              two launches per stage, the x-dimension terms of whole node
 *              rows, then the velocity terms of column blocks with the RK
 *              update (only xcd_remap and options bit 0 apply); 1 = the
 *              kernel specialised for d = 6 (3 x + 3 v) at degree 3, one cell
 *              per 256-thread workgroup (only xcd_remap and options apply;
 *              its FP64 first- and last-stage variants always take one slab
 *              per XCD). Under quadrature 1, or on mapped cells (see
 *              hd_set_mapping), it selects the kernel of the same layout for
 *              that discretization (Gauss-Legendre, mapped collocation or
 *              mapped Gauss-Legendre; xcd_remap and the streaming stores
 *              apply, except that mapped collocation always takes one slab
 *              per XCD).
 *  options:    bit 0 (every kernel): non-temporal (streaming) loads and
 *              stores of the stage increment du and stores of the output
 *              solution, so they do not displace cached neighbour data;
 *              bit 1 (kernel 1, FP32 only): keep the FP64 input solution in
 *              registers instead of re-reading it for the update (the
 *              generic kernel does so by itself when a thread owns at most
 *              8 nodes).
 *  split_dims: (kernel 0, lds = 1) number of velocity dimensions, just below
 *              the register dimensions, along which a cell is cut into slabs
 *              of one node layer each; a workgroup stages one slab in LDS and
 *              reads the other slabs of the line from global memory. 0, 1 or
 *              2; compiled for degree >= 4 at d >= 5, for cells too large to
 *              stage whole.
 *  loop_dims:  (kernel 0, lds = 1, cells_per_wg = 1) 1 = a thread covers the
 *              k+1 pencils that differ in the slowest thread-distributed
 *              dimension one after another, so units of more than 1024
 *              pencils fit a workgroup; compiled for degree >= 4 at d >= 5. */
typedef struct {
  int lds;
  int cells_per_wg;
  int wg_size;
  int xcd_remap;
  int reg_dims;
  int kernel;
  int options;
  int split_dims;
  int loop_dims;
} hd_plan;

/* Create a solver for `mesh` (the tensor-product mesh of Sec. 3.1, eq.
 * concept:tria:tensor) and polynomial degree `degree` (the nodal basis of
 * Sec. 2.3: k+1 Gauss-Lobatto nodes per dimension; degree 1..5 compiled)
 * with precision `prec` (hd_precision). The field defaults to constant
 * zero. Allocates no device memory; *out is NULL on error.
 * Errors: HD_ERR_INVALID (see the general conventions, or an unknown
 * precision); HD_ERR_UNSUPPORTED for degree > 5 or an x+v split other than
 * 1+1, 2+1, 2+2, 3+2, 3+3 (the splits of the paper's runs, Sec. 5.1). */
hd_status hd_create(const hd_mesh *mesh, int degree, int prec, hd_solver **out);

/* Destroy a solver: waits for its last captured RK step still in flight,
 * releases its host objects and graphs; the caller's bound memory is not
 * freed. NULL is a no-op. (Bookkeeping of this interface; no passage of the
 * paper.) */
hd_status hd_destroy(hd_solver *s);

/* Number of DoFs N = |C| (k+1)^d, the count of eq. dealii:totalunkonwns
 * (Sec. 2.3) for the tensor-product mesh. */
hd_status hd_num_dofs(const hd_solver *s, int64_t *ndofs);

/* Device memory the solver needs, in two caller-owned buffers. The
 * low-storage RK scheme of Sec. 5.4 keeps three solution-sized vectors:
 *  *state_bytes:     the state buffer, two FP64 solution vectors of N
 *                    values (the input and output of a fused stage, used in
 *                    turn; hd_state_ptr says which holds the solution);
 *  *workspace_bytes: the workspace, the stage increment du (N values, FP64
 *                    or FP32 by precision), the field table at the
 *                    configuration nodes, reduction partials, and for the
 *                    Vlasov-Poisson field or mapped cells their tables.
 * Each section is 256-byte aligned. Errors: HD_ERR_INVALID for NULL. */
hd_status hd_required_bytes(const hd_solver *s, size_t *state_bytes, size_t *workspace_bytes);

/* Hand the solver its caller-owned device memory: state_dev (at least
 * *state_bytes of hd_required_bytes) and workspace_dev (at least
 * *workspace_bytes), both 256-byte aligned and disjoint. The library never
 * frees them; they must outlive the solver's use. Both are cleared
 * (synchronously) and the solution starts as zero. Re-binding drops the
 * captured RK steps. Errors: HD_ERR_INVALID for NULL, short, misaligned or
 * overlapping buffers; HD_ERR_HIP if clearing fails. */
hd_status hd_bind(hd_solver *s, void *state_dev, size_t state_bytes, void *workspace_dev,
                  size_t workspace_bytes);

/* Constant advection field a (d entries) of eq. intro:advection (Sec. 1.2)
 * - the field of the paper's performance runs (Sec. 5.1). Synchronous if
 * bound (the table upload); before hd_bind it is kept and uploaded by
 * hd_bind. Errors: HD_ERR_INVALID for NULL or a non-finite entry. */
hd_status hd_set_field_constant(hd_solver *s, const double *a);

/* Phase-space field a = (v, sign * E(x)) (Sec. 1.2 eq. intro:vp:simple,
 * Sec. 6.1): a_{x_j} is the velocity coordinate v_j, a_{v_j} = sign*E_j(x).
 * E_host holds E at the configuration-space nodes,
 * E[((xcell * (k+1)^dx) + xnode) * dx + j], xcell and xnode lexicographic
 * (dim 1 fastest). Requires dim_x == dim_v. Copied to device; synchronous.
 * Requires hd_bind. */
hd_status hd_set_field_phase_space(hd_solver *s, const double *E_host, double sign);

/* Phase-space field (as hd_set_field_phase_space) with the prescribed
 * E_j(x) = amp * sin(2 pi (x_j - lo_j)/(hi_j - lo_j)) at the configuration
 * nodes: the synthetic stand-in for the field of Sec. 6.1 that the
 * benchmark workloads use. On mapped cells x is the mapped node position;
 * hd_set_mapping recomputes the table, so the two calls may come in either
 * order. Requires hd_bind and dim_x == dim_v. Synchronous. */
hd_status hd_set_field_sine(hd_solver *s, double amp, double sign);

/* Vlasov-Poisson field (Sec. 6, eq. vp:close): electrons on a neutralizing
 * background, a = (v, -E) with E recomputed from the input of every RK
 * stage (and of hd_apply) on the device, before the stage kernel, in the
 * same stream (and the same captured graph):
 *   rho(x) = int f dv            (GL quadrature over the velocity cells),
 *   -Laplace phi = 1 - rho,  E = -grad phi   on the periodic x-box,
 * solved spectrally: the Fourier coefficients of rho for the modes
 * |m_j| <= modes (exact discrete transforms over the GL nodes with the GL
 * weights), E_hat = i k rho_hat / |k|^2 (mode 0 dropped: the background
 * balances the mean), E = sum_m Re(E_hat e^{i k.x}) at the x-nodes.
 * The field is computed in FP64; FP32 solvers round it to FP32 for the
 * stage kernels. On C uniform cells the nodal pattern that repeats in every
 * cell transforms onto the modes that are multiples of C: for a physical
 * field keep modes below every x-dimension's cell count.
 * Requires dim_x == dim_v, 1 <= modes <= 16 and hd_bind.
 * Synchronous (uploads the transform matrices). */
hd_status hd_set_field_vlasov_poisson(hd_solver *s, int modes);

/* Copy the field table E to E_host (nE = (#x-cells)(k+1)^dx * dx doubles,
 * laid out as in hd_set_field_phase_space). For the Vlasov-Poisson field it
 * is first recomputed from the current state on `stream`; for a constant
 * field the table holds a_v at every x-node. Waits for `stream`. Requires
 * hd_bind and dim_x == dim_v. */
hd_status hd_get_field(hd_solver *s, double *E_host, hd_stream stream);

/* Quadrature of the DG integrals (Sec. 2.5): 0 = Gauss-Lobatto points
 * collocated with the nodes (diagonal mass matrix; the default), 1 =
 * Gauss-Legendre with k+1 points per dimension, the paper's default (the
 * exactly integrated mass matrix, applied through the basis change to the
 * Gauss points and back; a_v = E enters through the nodal interpolant of
 * the E table). The nodal GL basis and the state layout are the same for
 * both. Quadrature 1 runs one cell per workgroup with two cell-sized arrays
 * and a face layer in LDS and returns HD_ERR_UNSUPPORTED where those exceed
 * 160 KiB (FP64 6D degree >= 4, FP32 6D degree 5). For d = 6 (3 x + 3 v) at
 * degree 3 on Cartesian cells, plan kernel 1 (the default) selects a second
 * Gauss-Legendre kernel in the specialised kernel's thread layout (the same
 * operator, evaluated with 4 x 4 matrices in nodal space; xcd_remap
 * applies) and kernel 0 the general one; the other plan fields apply to
 * quadrature 0 only. */
hd_status hd_set_quadrature(hd_solver *s, int quadrature);

/* Curved configuration cells: the tensor-product mapping of Sec. 3.1 with a
 * deformed x-mesh and a Cartesian v-mesh. The box point X maps to
 *   x_m = X_m + eps (hi_m - lo_m) prod_{k < dim_x} sin(2 pi (X_k - lo_k)/(hi_k - lo_k)),
 * periodic, identity on the box faces. Node coordinates (initial states,
 * the sine field) follow the mapping; the operator is the weak form with
 * the contravariant flux |J| J^{-1} a at the quadrature points and the mass
 * matrix with |J|; the metric is stored at the x-quadrature points only
 * (per x-cell) and combined with the v-metric on the fly (Sec. 3.3).
 * Diagnostics weight with |J|. Works with either quadrature (one cell per
 * workgroup, as quadrature 1; for d = 6 (3 x + 3 v) at degree 3, plan
 * kernel 1, the default, runs either quadrature in the specialised
 * kernel's thread layout and kernel 0 the general one). eps = 0 restores Cartesian cells;
 * |eps| <= 0.05 (HD_ERR_INVALID otherwise, or if |J| <= 0 somewhere).
 * HD_ERR_UNSUPPORTED with the Vlasov-Poisson field, where the kernel's LDS
 * would exceed 160 KiB, and for 5D degree 5 (not compiled). The CFL estimate of hd_stable_dt ignores the
 * mapping. */
hd_status hd_set_mapping(hd_solver *s, double eps);

/* For the Vlasov-Poisson field: recompute the device E table from the
 * current state on `stream` (Sec. 6, steps 1-4 of a stage; asynchronous).
 * A no-op for prescribed fields. Requires hd_bind. */
hd_status hd_compute_field(hd_solver *s, hd_stream stream);

/* Copy a canonical FP64 state (N values; host or device pointer, as
 * u_is_device says) into the current solution buffer, on `stream`
 * (asynchronous; a host pointer must stay valid until the stream reaches
 * the copy). The nodal values are the coefficients of the nodal basis of
 * Sec. 2.3. Requires hd_bind. Errors: HD_ERR_INVALID for NULL or unbound. */
hd_status hd_set_state(hd_solver *s, const double *u, int u_is_device, hd_stream stream);

/* Nodal interpolation (values at the nodes of Sec. 2.3; the paper does not
 * say how initial data enter, this library interpolates) of an initial
 * state on the device, into the current solution buffer, on `stream`:
 *  kind 0: prod_j sin(2 pi (x_j - lo_j)/(hi_j - lo_j));
 *  kind 1: (1 + params[0] cos(2 pi (x_1 - lo_1)/(hi_1 - lo_1)))
 *          * (2 pi)^(-dv/2) exp(-|v|^2/2), the perturbed Maxwellian of the
 *          Landau-damping setting of Sec. 6.2.
 * Node positions follow the mapping on mapped cells. Requires hd_bind.
 * Errors: HD_ERR_INVALID for an unknown kind or unbound solver. */
hd_status hd_init_state(hd_solver *s, int kind, const double *params, hd_stream stream);

/* Device pointer to the current FP64 solution (N doubles, canonical),
 * inside the bound state buffer. It moves between the two solution vectors
 * after each RK stage (the ping-pong of the three-vector scheme, Sec. 5.4).
 * Requires hd_bind. */
hd_status hd_state_ptr(const hd_solver *s, void **dev_ptr);

/* Copy the current solution (canonical layout, Sec. 3.2 enumeration) to
 * host memory (N doubles) after the work queued on `stream`. Synchronizes
 * the stream. Requires hd_bind. */
hd_status hd_get_state(const hd_solver *s, double *u_host, hd_stream stream);

/* out = M^{-1} A(in): the element-centric evaluation of Algorithm 2 (cell
 * integral, 2d upwind face integrals, diagonal inverse mass) on every cell.
 * in: N FP64 values on the device (canonical, must not alias out);
 * out: N values on the device, FP64 for HD_FP64 and FP32 for HD_FP32. */
hd_status hd_apply(hd_solver *s, const double *in_dev, void *out_dev, hd_stream stream);

/* dt = cfl / ((2k+1) sum_j max|a_j| / h_j) for the current field. The
 * paper fixes no time-step rule (Sec. 5.4 names the scheme only); this is
 * the library's reading: the usual DG advective limit with the maximum of
 * |a_j| over the nodes, max|v_j| over the velocity nodes for a_{x_j} and
 * max|E_j| over the table for a_{v_j}. It ignores the mapping of mapped
 * cells. For the Vlasov-Poisson field, E is that of the current state,
 * computed on the null stream (which waits for blocking streams) before
 * this returns. Errors: HD_ERR_INVALID for cfl <= 0 or an all-zero field. */
hd_status hd_stable_dt(const hd_solver *s, double cfl, double *dt);

/* One stage (stage = 0..4) of the low-storage RK scheme (Sec. 5.4), fused
 * into one pass: du <- A_s du + dt M^{-1}A(u); u <- u + B_s du. Stages
 * 1..4 continue the step that stage 0 began: they read du, and under the
 * Vlasov-Poisson field with the 6D degree-3 kernel they take the density
 * from the velocity moments that the previous stage's kernel wrote with its
 * output (stage 0 always integrates the state itself). */
hd_status hd_rk_stage(hd_solver *s, int stage, double dt, hd_stream stream);

/* nsteps full RK steps (5 fused stages each), replayed from a hipGraph
 * captured per (dt, solution buffer parity). */
hd_status hd_rk_step(hd_solver *s, double dt, int nsteps, hd_stream stream);

/* The discrete mass and L2 energy of the current solution, integrated with
 * the Gauss-Lobatto quadrature of Sec. 2.5 (the diagonal mass matrix of the
 * collocated basis, Sec. 1.3): mass = sum_i W_i u_i, energy =
 * sum_i W_i u_i^2 with W_i = prod_j h_j w_{i_j} (times |J| at the node on
 * mapped cells). The upwind scheme conserves the first and does not
 * increase the second (Sec. 1.3). FP64 with a fixed reduction order
 * (bitwise reproducible); the partial sums live in the workspace.
 * Synchronizes `stream`. Requires hd_bind. */
hd_status hd_diagnostics(const hd_solver *s, double *mass, double *energy, hd_stream stream);

/* hd_diagnostics for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same two reduction kernels, in the same fixed order (bitwise equal to
 * hd_diagnostics on the same vector), with the partial sums in a
 * file-scope device array of the library instead of the workspace.
 *   s        a created solver (it need not be bound): mesh, degree, mapping;
 *   u_dev    FP64 device vector of hd_num_dofs values, canonical layout;
 *   res_dev  device memory for 2 doubles: res_dev[0] = mass,
 *            res_dev[1] = energy (written by a kernel on `stream`).
 * Enqueues two kernels on `stream` and returns; calls no allocating
 * routine and does not synchronize. The array holds 1024 partial pairs
 * (16 KiB per GPU, kept until the process ends); every call on one GPU
 * shares it, so calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller. Limit: at most 2^40
 * DoFs, else HD_ERR_INVALID; NULL arguments give HD_ERR_INVALID. */
hd_status hd_diagnostics_noalloc(const hd_solver *s, const double *u_dev, double *res_dev,
                                 hd_stream stream);

/* Read / override the stage-kernel launch plan (hd_plan above). Plans
 * change how the kernels map cells and nodes onto the GPU, never the
 * result beyond rounding order; they have no counterpart in the paper,
 * whose CPU code fixes its vectorization over cells (Sec. 4). hd_set_plan
 * returns HD_ERR_INVALID (with the reason) for a plan that does not fit
 * the limits or has no compiled kernel, and drops the captured steps. */
hd_status hd_get_plan(const hd_solver *s, hd_plan *plan);
hd_status hd_set_plan(hd_solver *s, const hd_plan *plan);

/* dst[i] = src[i], i < n, on the stream: a plain streaming copy used to
 * measure achievable HBM bandwidth and to calibrate byte counters (a
 * measurement aid; no passage of the paper). src and dst: device, 16-byte
 * aligned, not overlapping. */
hd_status hd_stream_copy(const double *src, double *dst, size_t n, hd_stream stream);

/* Message of the last error on this thread ("" if none); the pointer stays
 * valid until the thread's next failing call. (Bookkeeping of this
 * interface; no passage of the paper.) */
const char *hd_last_error(void);

/* Batched stepping of many independent solves (Sec. 5.4 time stepping of
 * each; any d, degree, size, precision and plan in one batch).
 * hd_batch_step advances every active solve by one LSRK step with ONE
 * hipGraph replay. Per RK stage, the solves whose stage kernel has a
 * work-list form (collocation on Cartesian cells with a prescribed field)
 * are grouped by kernel variant and launch shape, and each group is ONE
 * launch over a work list of (solve, tile) items, one workgroup per item,
 * running the solve's own stage body with its own parameters; the others
 * (Gauss-Legendre, mapped cells, the Vlasov-Poisson field, or a variant
 * whose work-list form would hold fewer workgroups per CU or more scratch
 * than its own launch) keep their own stage launches in the same graph.
 * Either way a solve's result is bitwise the same alone and in the batch.
 * The kernel parameters and work lists are built and checked on the host,
 * uploaded into device memory of the batch before the graph is captured,
 * and freed only after that graph's last replay. The graph is captured at
 * the first step and again whenever the active set, a time step, a
 * solution-buffer parity or a solver's plan, field or memory changed; two
 * graphs are cached (alternating parities).
 * Ownership: `solvers` (n pointers, read during the call) stay owned by the
 * caller, must stay bound and outlive the batch; destroying or re-binding
 * a member while the batch is used is undefined.
 * Errors: HD_ERR_INVALID for NULL arguments, n outside 1..1024, an unbound
 * solver or one listed twice; HD_ERR_OOM; HD_ERR_HIP if stream, event or
 * graph set-up fails. */
hd_status hd_batch_create(hd_solver *const *solvers, int n, hd_batch **out);
hd_status hd_batch_destroy(hd_batch *b);

/* One RK step of every solver i with active[i] != 0 (active = NULL: all),
 * with time step dt[i] (host arrays of n entries; dt is ignored for
 * inactive solves). Enqueued on `stream`, asynchronous; nothing is launched
 * if no solve is active. Each active solver's solution ends in its other
 * buffer (hd_state_ptr follows). Calls that overlap on one solver race.
 * Errors: HD_ERR_INVALID for NULL b or dt, a non-finite dt of an active
 * solve, or a member that lost its workspace; HD_ERR_HIP for capture or
 * launch failures. */
hd_status hd_batch_step(hd_batch *b, const double *dt, const int *active, hd_stream stream);

/* Launches in the most recently captured step of b: work-list launches (one
 * per kernel-variant group and stage) and stage launches of single solves.
 * Both 0 before the first step. (Bookkeeping of this interface.)
 * Errors: HD_ERR_INVALID for NULL arguments. */
hd_status hd_batch_launch_counts(const hd_batch *b, int *list_launches, int *solve_launches);

#ifdef __cplusplus
}
#endif
#endif /* HD_H */
