/*
 * egfem.h -- C ABI of libegfem, the MI355X (gfx950) EGFEM Newton hot path.
 *
 * Method: Tolle & Marheineke, "Extended Group Finite Element Method"
 * (arXiv 2005.06193).  A nonlinear coefficient a(u) is interpolated onto its
 * own space W_h (here W_h = V_h = P1, Case 2 of Sec. 3.1, i.e. the group FEM
 * choice), so the nonlinear form becomes the trilinear form of eq.
 * (egfem_terms):
 *
 *     (K_a : (u (x) a))_i = sum_jk T_ijk u_j a_k,
 *     T_ijk = int phi_k grad phi_j . grad phi_i      (EGFEM_FORM_STIFF)
 *     T_ijk = int phi_k phi_j phi_i                  (EGFEM_FORM_MASS, the
 *             trilinear mass form of Sec. 5.3, decomposition (a)),
 *     T_ijk = int phi_k phi_j sum_d d_d phi_i        (EGFEM_FORM_CONV, the
 *             convection tensor N of Burgers' equation, Sec. 5.2).
 *
 * The discrete problem solved is the u-reduced form of eq. (EGFEM_root):
 *
 *     F(u) = [K u] + T:(u (x) a(u)) - d = 0   on the free nodes,
 *     a(u) = a0 + u*u (pointwise at the nodes, eq. egfem_coeffs, Pi_u = I),
 *     u = 0 on the Dirichlet nodes,
 *
 * by Newton's method (Sec. 4).  Its Jacobian needs no integration, only the
 * contractions of the Notation in Sec. 3.3:
 *
 *     DF = [K] + T . a + (T ._2 u) diag(a'(u)),   a'(u) = 2u,
 *
 * emitted into the fixed CSR pattern of the P1 node adjacency (diagonal
 * included) and solved with preconditioned BiCGStab (block-Jacobi on compact
 * row parts, or Jacobi: the launch shape's krylov_precond).
 *
 * Conventions for every entry point below
 *  - Vectors are float64 and contiguous.  Pointers documented as "device" are
 *    HIP device pointers owned by the caller (e.g. torch tensor storage); the
 *    library never frees them.  "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    kernels of a call are enqueued on it.  Calls that return numbers to the
 *    host (norms, statistics) synchronise that stream; the others do not.
 *  - Return value: 0 = EGFEM_OK; > 0 = numerical outcome (outputs and
 *    statistics are valid); < 0 = error, nothing was written, and
 *    egfem_last_error() returns a message (thread-local).
 *  - A handle owns the device buffers it allocates (tensor streams, pattern,
 *    matrices, solver workspace).  Calls that use the solver workspace of a
 *    handle (newton, solve) must not run concurrently on the same handle.
 *  - Results are deterministic for a fixed launch configuration: no floating
 *    point atomics; reductions use a fixed order.
 */
#ifndef EGFEM_H
#define EGFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct egfem_tensor_s* egfem_tensor_t;

enum egfem_status {
  EGFEM_OK = 0,
  EGFEM_NOT_CONVERGED = 1,   /* iteration cap reached */
  EGFEM_BREAKDOWN = 2,       /* BiCGStab breakdown (rho or omega ~ 0) after one restart */
  EGFEM_NONFINITE = 3,       /* NaN/Inf met in a residual or Krylov scalar */
  EGFEM_STAGNATED = 4,       /* no damped step decreases ||F|| (rounding floor reached) */
  EGFEM_ERR_ARG = -1,        /* null pointer, bad enum, bad option value */
  EGFEM_ERR_SHAPE = -2,      /* sizes inconsistent or beyond a documented limit */
  EGFEM_ERR_OOM = -3,        /* device or host allocation failed */
  EGFEM_ERR_HIP = -4,        /* a HIP runtime call failed */
  EGFEM_ERR_MESH = -5        /* cell index out of range or degenerate simplex */
};

enum egfem_form {
  EGFEM_FORM_STIFF = 0,      /* T_ijk = int phi_k grad phi_j . grad phi_i */
  EGFEM_FORM_MASS = 1,       /* T_ijk = int phi_k phi_j phi_i (fully symmetric) */
  EGFEM_FORM_CONV = 2        /* T_ijk = int phi_k phi_j (sum_d d/dx_d phi_i) (T_ijk = T_ikj) */
};

enum egfem_wspace {
  EGFEM_W_P1 = 0,            /* W_h = V_h = P1 (Case 2 of Sec. 3.1, the group FEM choice) */
  EGFEM_W_P2 = 1,            /* W_h = P2 on the same mesh with Pi_u the P2 interpolation of the
                                P1 iterate (Case 1 of Sec. 3.1): for a = a0 + u^2 the coefficient
                                is then exact and EGFEM coincides with the standard Galerkin method */
  EGFEM_W_IQ = 2,            /* W_h = I_k (Case 3 of Sec. 3.1): the coefficient lives at the points
                                of a fixed quadrature rule in every cell (1D: 2-point Gauss; 2D: the
                                3 points with barycentrics (2/3,1/6,1/6); 3D: the 4 points (a,b,b,b),
                                a = (5+3 sqrt 5)/20, b = (5-sqrt 5)/20; equal weights), Pi_u evaluates
                                the P1 iterate there; the stiffness form is then again exact */
  EGFEM_W_P0 = 3             /* W_h = P0 (one dof per cell) for nonlinearities of the gradient
                                (Sec. 3.2, the p-Laplace and minimal surface examples of Sec. 5):
                                T_ijk = K^{e_k}_ij (stiffness) or M^{e_k}_ij (mass); the
                                coefficient comes from egfem_picard_grad or is passed per cell */
};

/* ------------------------------------------------------------------------
 * Offline phase (Sec. 3.3 eq. egfem_terms; the paper excludes it from the
 * online times, Sec. 5 preamble).
 *
 * egfem_build_tensor: assemble T, the P1 stiffness matrix K_ij = int grad
 * phi_j . grad phi_i and the consistent mass matrix M_ij = int phi_j phi_i on
 * a conforming P1 simplex mesh, by exact integration of the element
 * polynomials, and upload them as device streams.
 *   dim      1, 2 or 3
 *   coords   host [n_nodes * dim], node-major (x0,y0,x1,y1,...)
 *   cells    host [n_cells * (dim+1)], 0-based node ids of each simplex
 *   form     EGFEM_FORM_STIFF, EGFEM_FORM_MASS or EGFEM_FORM_CONV
 *   drop_rel after summing element contributions, an entry is dropped when
 *            |T_ijk| <= drop_rel * max_{j',k'} |T_ij'k'| (0: only exact zeros).
 *            1e-13 removes the entries that vanish in exact arithmetic.
 *   out      receives the handle.
 * Limits: n_nodes < 2^31, stored entries < 2^31, and every node row must fit
 * one row block (<= 1024 tensor entries and <= 512 adjacency slots per row),
 * else EGFEM_ERR_SHAPE.  A zero-volume cell or an index outside [0, n_nodes)
 * gives EGFEM_ERR_MESH.  Synchronous (host arrays may be reused on return).
 * ---------------------------------------------------------------------- */
int egfem_build_tensor(int dim, int64_t n_nodes, const double* coords,
                       int64_t n_cells, const int32_t* cells, int form,
                       double drop_rel, egfem_tensor_t* out);

/* egfem_build_tensor_w: the same with the coefficient space chosen by wspace.
 * With EGFEM_W_P2 the tensor is T_ijk = int eta_k grad phi_j . grad phi_i
 * (stiffness) or int eta_k phi_j phi_i (mass) with eta the P2 nodal basis
 * (vertex lambda(2 lambda - 1), edge midpoint 4 lambda_x lambda_y), or
 * int eta_k phi_j sum_d d_d phi_i (convection, for egfem_burgers); k runs
 * over the n_w = n_nodes + n_edges P2 dofs: the vertices, then the edges in
 * ascending (smaller vertex id, larger vertex id) order (Sec. 3.1, Case 1;
 * Sec. 3.2 for Pi_u).  With EGFEM_W_IQ, k = e * Q + q runs over the Q points
 * of every cell e (n_w = n_cells * Q) and T_ijk = w_q |e| grad phi_j . grad
 * phi_i (stiffness), w_q |e| phi_j(x_q) phi_i(x_q) (mass) or w_q |e|
 * phi_j(x_q) sum_d d_d phi_i (convection, for egfem_burgers), (Pi_u u)_k =
 * u_h(x_q) (Sec. 3.1, Case 3).  On such a handle:
 *  - every a / dadu argument of egfem_residual and egfem_jacobian is a vector
 *    over the dofs of W_h (length n_w), and the second Jacobian term becomes
 *    sum_k (sum_j' T_ij'k u_j') dadu_k (Pi_u)_kj;
 *  - the problem-level calls (problem residual / Jacobian, Newton, Picard)
 *    use a = Pi_u a0 + (Pi_u u)^2 at the dofs of W_h, a' = 2 Pi_u u;
 *  - egfem_mode3, egfem_adjoint and the batched form return EGFEM_ERR_ARG;
 *    egfem_burgers takes a W_h = P2 or I_k convection handle with group = 1
 *    only; the convection form with EGFEM_W_P0 is EGFEM_ERR_ARG;
 *  - with EGFEM_W_P0 (k = cell, T_ijk = K^{e_k}_ij or M^{e_k}_ij) the problem-
 *    level calls return EGFEM_ERR_ARG (the coefficient is a function of the
 *    gradient: egfem_picard_grad), and egfem_jacobian takes no dadu.
 * Row blocks additionally hold at most 1024 (row, W_h dof) couplings. */
int egfem_build_tensor_w(int dim, int64_t n_nodes, const double* coords,
                         int64_t n_cells, const int32_t* cells, int form, int wspace,
                         double drop_rel, egfem_tensor_t* out);

void egfem_tensor_destroy(egfem_tensor_t T);

/* Sizes and read-only device views of the pattern (for callers that build
 * their own matrices in the same CSR pattern). */
typedef struct {
  int dim;
  int form;
  int symmetric;             /* 1: T_ijk = T_ikj (mass, convection), the B-stream aliases A */
  int64_t n_nodes;
  int64_t n_cells;
  int64_t nnz;               /* stored entries of T (A-stream length) */
  int64_t nnz_b;             /* B-stream length (== nnz) */
  int64_t structural_nnz;    /* entries before the drop rule */
  int64_t slots;             /* CSR entries of the P1 adjacency incl. diagonal */
  int64_t row_blocks;        /* row blocks of the tensor-action kernels */
  int64_t device_bytes;      /* bytes of device memory owned by the handle */
  const int32_t* rowptr;     /* device [n_nodes+1] */
  const int32_t* col;        /* device [slots], ascending within a row */
  const double* kval;        /* device [slots] stiffness matrix values */
  const double* mval;        /* device [slots] mass matrix values */
  int wspace;                /* EGFEM_W_P1, EGFEM_W_P2, EGFEM_W_IQ or EGFEM_W_P0 */
  int64_t n_w;               /* dofs of W_h (n_nodes for P1) */
  int64_t nnz_half;          /* entries of the symmetric half stream (0: none) */
} egfem_info;

int egfem_tensor_info(egfem_tensor_t T, egfem_info* info);

/* Copy the stored tensor to host COO arrays, ordered by (i, j, k), each of
 * length info.nnz (caller-allocated host memory).  Synchronous. */
int egfem_tensor_export(egfem_tensor_t T, int32_t* i, int32_t* j, int32_t* k, double* v);

/* Copy the CSR pattern to host arrays rowptr [n_nodes+1] and col [slots]
 * (caller-allocated).  Synchronous. */
int egfem_tensor_pattern(egfem_tensor_t T, int32_t* rowptr, int32_t* col);

/* ------------------------------------------------------------------------
 * Online tensor actions (Notation of Sec. 3.3).
 * ---------------------------------------------------------------------- */

/* egfem_residual: raw trilinear action r_i = sum_jk T_ijk u_j a_k
 * (second contraction T:(u (x) a), eq. egfem_terms).  No boundary rows, no
 * load.  u, a, r: device [n_nodes]; r must not alias u or a. */
int egfem_residual(egfem_tensor_t T, const double* u, const double* a, double* r,
                   void* stream);

/* ------------------------------------------------------------------------
 * Element-factored form of the stiffness tensor (storage comparison): with P1
 * coefficient functions and constant gradients, T^e_ijk = K^e_ij / (d+1) on
 * every cell, so
 *     (T:(u (x) a))_i = sum_{e contains i} abar_e (K^e u_e)_i,  abar_e = mean of a on e.
 * egfem_attach_elements stores, for an EGFEM_FORM_STIFF handle with W_h = P1,
 * the cells (4 ids each), the packed symmetric K^e and the node -> cell
 * incidence (cell id, local index) of the same mesh; the stream format is kept.
 *   coords, cells: host, as for egfem_build_tensor (must be the same mesh).
 * Returns EGFEM_ERR_ARG for another form or coefficient space, EGFEM_ERR_SHAPE
 * when the sizes differ from the handle's, EGFEM_ERR_MESH for bad cells.
 * Synchronous.  Attaching twice replaces the data. */
int egfem_attach_elements(egfem_tensor_t T, int dim, int64_t n_nodes, const double* coords,
                          int64_t n_cells, const int32_t* cells);

/* egfem_residual_elementwise: r = T:(u (x) a) through the element-factored
 * form (equal to egfem_residual up to rounding).  u, a, r: device [n_nodes],
 * r must not alias u or a.  EGFEM_ERR_ARG when no elements are attached. */
int egfem_residual_elementwise(egfem_tensor_t T, const double* u, const double* a, double* r,
                               void* stream);

/* ------------------------------------------------------------------------
 * Unique storage of the fully symmetric mass tensor (storage comparison; the
 * storage cost of the tensors is the trade-off noted in Sec. 5.5).  The P1 mass
 * tensor T_ijk = int phi_i phi_j phi_k (Sec. 3.3) is invariant under every
 * permutation of (i, j, k), so one value per index multiset suffices: T_iii per
 * node, T_aab and T_abb per edge (a < b) and T_abc per face (three distinct
 * vertices of a cell), N + 2E + F values instead of the N + 6E + 6F entries of
 * the stream.  The action gathers them per row:
 *     r_i = T_iii u_i a_i + sum_{j ~ i} [T_iij (u_i a_j + u_j a_i) + T_ijj u_j a_j]
 *         + sum_{faces {i,j,k}} T_ijk (u_j a_k + u_k a_j).
 * egfem_attach_unique stores, for an EGFEM_FORM_MASS handle with W_h = P1, the
 * values (integrated from the same mesh), per slot of the handle's pattern its
 * edge, and per row its faces with the row-local slots of their other two
 * vertices; the stream format is kept.
 *   coords, cells: host, as for egfem_build_tensor (must be the same mesh).
 *   n_unique (host, nullable) receives N + 2E + F.
 * Returns EGFEM_ERR_ARG for another form or coefficient space, EGFEM_ERR_SHAPE
 * when the mesh does not give the handle's sizes, entry count or pattern (or a
 * row has more than 512 slots), EGFEM_ERR_MESH for bad cells.  Synchronous.
 * Attaching twice replaces the data. */
int egfem_attach_unique(egfem_tensor_t T, int dim, int64_t n_nodes, const double* coords,
                        int64_t n_cells, const int32_t* cells, int64_t* n_unique);

/* egfem_residual_unique: r = T:(u (x) a) through the unique storage (equal to
 * egfem_residual up to rounding; deterministic).  u, a, r: device [n_nodes], r
 * must not alias u or a.  EGFEM_ERR_ARG when no unique storage is attached. */
int egfem_residual_unique(egfem_tensor_t T, const double* u, const double* a, double* r, void* stream);

/* egfem_jacobian: emit J in the CSR pattern of T (Sec. 4, block Jacobian
 * reduced to u; no integration):
 *   J_ij = [K_ij] + sum_k T_ijk a_k + dadu_j * sum_j' T_ij'j u_j'
 * u, a: device [n_nodes]; dadu: device [n_nodes] or NULL (term omitted);
 * add_stiffness: nonzero adds K; dirichlet: device uint8 [n_nodes] or NULL --
 * rows with dirichlet[i] != 0 become identity rows and columns of such nodes
 * become zero in the other rows; jval: device [slots].  dinv: device
 * [n_nodes] or NULL, receives 1 / J_ii (Jacobi preconditioner). */
int egfem_jacobian(egfem_tensor_t T, const double* u, const double* a, const double* dadu,
                   int add_stiffness, const uint8_t* dirichlet, double* jval, double* dinv,
                   void* stream);

/* egfem_mode3: out_k = sum_ij w_i T_ijk u_j (adjoint of the a-dependence of
 * the residual, i.e. ((T ._2 u)^T w)_k).  w, u, out: device [n_nodes]. */
int egfem_mode3(egfem_tensor_t T, const double* w, const double* u, double* out, void* stream);

/* egfem_matvec: y = A x for a matrix in T's CSR pattern.
 * which: 0 = jval (caller values, device [slots]), 1 = stiffness K, 2 = mass M.
 * transpose: nonzero computes A^T x (through the slot transpose permutation;
 * deterministic, no atomics).  x, y: device [n_nodes], no aliasing. */
int egfem_matvec(egfem_tensor_t T, int which, const double* jval, int transpose,
                 const double* x, double* y, void* stream);

/* ------------------------------------------------------------------------
 * The nonlinear problem and Newton's method (Sec. 4).
 * ---------------------------------------------------------------------- */
typedef struct {
  const double* a0;          /* device [n_nodes] or NULL: then a0_const everywhere */
  double a0_const;
  const double* load;        /* device [n_nodes]: the load vector d (e.g. M f) */
  const uint8_t* dirichlet;  /* device [n_nodes], nonzero = Dirichlet node (u = 0); NULL = none */
  int add_stiffness;         /* nonzero: F gets + K u (semilinear form) */
} egfem_problem;

/* F = [K u] + T:(u (x) (a0 + u*u)) - d, Dirichlet rows 0.  u, F: device.
 * If norm != NULL it receives ||F||_2 on the host (synchronises the stream). */
int egfem_problem_residual(egfem_tensor_t T, const egfem_problem* p, const double* u,
                           double* F, double* norm, void* stream);

/* egfem_problem_residual_noalloc: egfem_problem_residual for callers that
 * cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments and result (F
 * bitwise equal; the norm's partial sums are added in another fixed order).
 * Allocates nothing: the residual kernel's per-workgroup partial sums and
 * their total live in a fixed array of the library (one per device, held
 * until the process ends, 16,384 partial sums = 128 KiB); the total is formed
 * on the device and, with norm != NULL, copied to *norm (synchronises the
 * stream).  The handle's device must be current.  EGFEM_ERR_SHAPE when the
 * handle's residual kernel writes more than 16,384 partial sums (an untuned
 * handle writes one per row block; autotuned action runs write at most 8,192).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller. */
int egfem_problem_residual_noalloc(egfem_tensor_t T, const egfem_problem* p, const double* u,
                                   double* F, double* norm, void* stream);

/* DF(u) = [K] + T . a + (T ._2 u) diag(2u) with Dirichlet identity rows and
 * zero Dirichlet columns, into jval (device [slots]); dinv optional as above. */
int egfem_problem_jacobian(egfem_tensor_t T, const egfem_problem* p, const double* u,
                           double* jval, double* dinv, void* stream);

typedef struct {
  double tol;                /* stop when ||F||_2 <= tol * ||F(u0)||_2 (default 1e-10) */
  int max_newton;            /* default 50 */
  int max_krylov;            /* BiCGStab iterations per linear solve (default 20000) */
  double krylov_rtol;        /* inner relative tolerance when forcing == 0 (default 1e-12) */
  int forcing;               /* 0: fixed krylov_rtol; 1: Eisenstat-Walker choice 2 */
  double eta_max;            /* EW cap (default 0.1) */
  int max_backtracks;        /* damping halvings (default 10) */
  int krylov_blocks;         /* persistent Krylov grid size, 0 = the handle's launch shape */
  int krylov_threads;        /* persistent Krylov workgroup size: 256, 512 or 1024, 0 = the
                                handle's launch shape */
  int timing;                /* nonzero: time every kernel launch with HIP events on the
                                stream (fills the t_* / n_* fields of the statistics) */
} egfem_newton_opts;

#define EGFEM_HIST 64

typedef struct {
  int status;                /* egfem_status of the solve */
  int newton_iters;
  int krylov_iters;          /* total over all Newton steps */
  int backtracks;
  double res0;               /* ||F(u0)||_2 */
  double res;                /* final ||F||_2 */
  double res_hist[EGFEM_HIST];    /* ||F|| after step k (k < EGFEM_HIST) */
  int krylov_hist[EGFEM_HIST];    /* Krylov iterations of step k */
  /* with opts.timing: summed launch durations (ms) and launch counts */
  double t_action_ms;        /* fused residual / trial-iterate tensor action */
  double t_jacobian_ms;      /* Jacobian emission */
  double t_krylov_ms;        /* persistent BiCGStab */
  int n_action;
  int n_jacobian;
  int n_krylov;
  int krylov_status_hist[EGFEM_HIST];     /* Krylov status of step k */
  double krylov_relres_hist[EGFEM_HIST];  /* Krylov relative residual of step k */
  int krylov_kernels;        /* BiCGStab kernels that ran: bit 0 register-resident, bit 1 streaming,
                                bit 2 with the block-Jacobi preconditioner, bit 3 the overlapped
                                form (flag-in-data synchronisation, see krylov_kernel) */
} egfem_newton_stats;

/* Fill opts with the defaults above. */
void egfem_newton_opts_default(egfem_newton_opts* o);

/* egfem_newton: damped Newton from the guess in u (device [n_nodes]; Dirichlet
 * entries are set to 0) to the solution, written back into u.  A step
 * u + alpha delta is accepted when ||F|| <= (1 - 1e-4 alpha) ||F(u)||, halving
 * alpha up to max_backtracks times; if none passes, status EGFEM_STAGNATED and
 * u is the last accepted iterate.  Per step: fused residual + norm, Jacobian
 * emission, one persistent BiCGStab launch; the host reads back two scalars per
 * step.  s may be NULL.  Synchronises the stream. */
int egfem_newton(egfem_tensor_t T, const egfem_problem* p, double* u,
                 const egfem_newton_opts* o, egfem_newton_stats* s, void* stream);

/* egfem_solve: preconditioned BiCGStab (krylov_precond) for A x = rhs, A = J (jval in
 * T's pattern) or J^T (transpose != 0).  x: device, initial guess on input.
 * Stops when ||rhs - A x||_2 <= rtol ||rhs||_2 (recursive residual) or after
 * max_iter iterations.  iters / relres (host, nullable) receive the outcome.
 * Returns EGFEM_OK, EGFEM_NOT_CONVERGED, EGFEM_BREAKDOWN or EGFEM_NONFINITE.
 * Synchronises the stream. */
int egfem_solve(egfem_tensor_t T, const double* jval, int transpose, const double* rhs,
                double* x, double rtol, int max_iter, int* iters, double* relres, void* stream);

/* ------------------------------------------------------------------------
 * Picard iteration (Sec. 4, Example picard_iteration): the previous iterate
 * is substituted into the nonlinear coefficient and the linear system
 *     ([K] + T . a(u^n)) u^{n+1} = d,   a(u^n) = a0 + (u^n)^2 pointwise,
 * is solved for the new iterate; Dirichlet rows are identity rows with zero
 * right-hand side.  The matrix is the A-stream emission of egfem_jacobian
 * without the a' term; it is symmetric positive definite on the free rows,
 * so the linear solves are preconditioned conjugate gradients (krylov_precond)
 * (single-reduction arrangement, one persistent cooperative launch), warm
 * started from u^n.
 * ---------------------------------------------------------------------- */
typedef struct {
  double tol;                /* stop when ||u^{n+1} - u^n||_2 <= tol ||u^{n+1}||_2 (default 1e-12) */
  int max_picard;            /* iteration cap (default 200) */
  int max_krylov;            /* CG iteration cap per solve (default 20000) */
  double krylov_rtol;        /* each solve: ||r|| <= krylov_rtol ||r_0|| with r_0 = d - A(u^n) u^n,
                                i.e. relative to the nonlinear residual of u^n (default 0.1: inexact
                                steps; the tolerance tightens with the residual) */
  int krylov_blocks;         /* persistent CG grid size, 0 = launch shape of the handle */
  int krylov_threads;        /* 256, 512, 1024, or 0 = launch shape of the handle */
  int timing;                /* nonzero: time the matrix emissions and solves with HIP events */
} egfem_picard_opts;

typedef struct {
  int status;                /* EGFEM_OK, EGFEM_NOT_CONVERGED or EGFEM_NONFINITE */
  int picard_iters;
  int krylov_iters;          /* total CG iterations */
  double update;             /* last relative update ||u^{n+1} - u^n|| / ||u^{n+1}|| */
  double res0;               /* ||F(u_0)||_2 over the free rows */
  double res;                /* ||F(u)||_2 at the returned iterate */
  double update_hist[EGFEM_HIST];
  int krylov_hist[EGFEM_HIST];
  double t_matrix_ms;        /* with timing: matrix emissions */
  double t_krylov_ms;        /* with timing: CG launches */
  int krylov_kernels;        /* CG kernels that ran: bit 0 register-resident, bit 1 streaming */
} egfem_picard_stats;

/* Fill opts with the defaults above. */
void egfem_picard_opts_default(egfem_picard_opts* o);

/* egfem_picard: Picard iteration from the guess in u (device [n_nodes];
 * Dirichlet entries are set to 0) to the fixed point, written back into u.
 * p as for egfem_newton; its a0 / a0_const / load / add_stiffness define F.
 * s (host, nullable) receives the statistics.  Returns the status (EGFEM_OK
 * when the update test passed) or a negative error.  Synchronises the stream. */
int egfem_picard(egfem_tensor_t T, const egfem_problem* p, double* u, const egfem_picard_opts* o,
                 egfem_picard_stats* s, void* stream);

/* egfem_solve_cg: preconditioned conjugate gradients (krylov_precond) for A x = rhs with
 * A (jval, T's pattern) symmetric positive definite, e.g. the matrix of a
 * Picard step.  x: device, initial guess on input, solution on output.  Stops
 * when ||rhs - A x||_2 <= rtol ||rhs||_2 (recursive residual) or after max_iter
 * iterations; iters / relres (host, nullable) receive the outcome.  Returns
 * EGFEM_OK, EGFEM_NOT_CONVERGED, EGFEM_BREAKDOWN (a non-positive curvature, so
 * A is not SPD) or EGFEM_NONFINITE.  Synchronises the stream. */
int egfem_solve_cg(egfem_tensor_t T, const double* jval, const double* rhs, double* x, double rtol,
                   int max_iter, int* iters, double* relres, void* stream);

/* ------------------------------------------------------------------------
 * Viscous Burgers' equation, semi-implicit time stepping (Sec. 5.2):
 *     u_t - nu Lap u + u sum_d d_d u = d,   u = 0 on the Dirichlet nodes.
 * With u sum_d d_d u = 1/2 sum_d d_d (u^2) and integration by parts, each step
 * takes the nonlinear term at the old time level and solves
 *     (M + dt nu K) u^{n+1} = M (u^n + dt s^{n+1}) + dt/2 C(u^n),
 *     C(u) = N:(u (x) u)                        (group = 0, tensor formulation),
 *     C(u) = N^f (u . u), N^f_ik = sum_j N_ijk  (group = 1, group formulation:
 *            u^2 interpolated onto P1; N^f is int phi_k sum_d d_d phi_i),
 *     C(u) = N^f_P2 (Pi_u u)^2                  (group = 1 on a W_h = P2 handle:
 *            the EGFEM group formulation, N^f_P2 = int eta_k sum_d d_d phi_i,
 *            (Pi_u u)^2 squared at the P2 dofs; equal to the tensor
 *            formulation up to rounding, since u^2 of a P1 u lies in P2),
 *     C(u) = N^f_I (Pi_u u)^2                   (group = 1 on a W_h = I_k handle:
 *            N^f_I,ik = w_q |e| sum_d d_d phi_i for k = (e, q), u_h squared
 *            at the points; equal to the tensor formulation up to rounding
 *            where the rule integrates the quadratic u_h^2 exactly, which
 *            the rules of EGFEM_W_IQ do),
 * with N the EGFEM_FORM_CONV tensor of the handle, s^{n+1} the nodal source
 * values at t_{n+1} (load M s^{n+1}), Dirichlet rows identity with zero right-
 * hand side.  The matrix is constant and symmetric positive definite: it is
 * emitted once, and every step is one tensor action (or one N^f product fused
 * into the right-hand side) plus one persistent preconditioned CG launch started from
 * an extrapolation of the previous iterates (opts.guess).
 * ---------------------------------------------------------------------- */
typedef struct {
  double dt;                 /* time step (default 1e-2) */
  double nu;                 /* viscosity (default 1) */
  int steps;                 /* number of steps (default 100) */
  int group;                 /* 0: tensor formulation, 1: group formulation (default 0) */
  double krylov_rtol;        /* each solve: ||r||_2 <= krylov_rtol ||rhs||_2 (default 1e-12) */
  int max_krylov;            /* CG iteration cap per step (default 20000) */
  int guess;                 /* initial CG iterate of step n+1: 0 = u^n, 1 = 2u^n - u^{n-1},
                                2 = 3u^n - 3u^{n-1} + u^{n-2} (polynomial extrapolation in time,
                                lower order while fewer iterates exist; default 2) */
  int krylov_blocks;         /* persistent CG grid, 0 = launch shape of the handle */
  int krylov_threads;        /* 256, 512, 1024, or 0 = launch shape of the handle */
  int timing;                /* nonzero: time the right-hand sides and solves with HIP events */
} egfem_burgers_opts;

typedef struct {
  int status;                /* worst step status: EGFEM_OK, NOT_CONVERGED, BREAKDOWN or NONFINITE */
  int steps;                 /* steps taken (fewer than asked only after a non-finite step) */
  int64_t krylov_iters;      /* total CG iterations */
  int max_step_krylov;       /* most CG iterations of one step */
  double max_relres;         /* largest final relative CG residual of a step */
  int krylov_hist[EGFEM_HIST];    /* CG iterations of step n (n < EGFEM_HIST) */
  double t_rhs_ms;           /* with timing: tensor actions and right-hand sides */
  double t_krylov_ms;        /* with timing: CG launches */
  int krylov_kernels;        /* CG kernels that ran: bit 0 register-resident, bit 1 streaming */
} egfem_burgers_stats;

/* Fill opts with the defaults above. */
void egfem_burgers_opts_default(egfem_burgers_opts* o);

/* egfem_burgers: advance u (device [n_nodes], u^0 in, u^steps out; Dirichlet
 * entries are set to 0) by opts->steps semi-implicit steps.  T must be an
 * EGFEM_FORM_CONV handle (its K and M are the stiffness and mass matrices);
 * a W_h = P2 or I_k handle needs opts->group = 1 (EGFEM_ERR_ARG otherwise).
 *   dirichlet      device uint8 [n_nodes] or NULL (no Dirichlet nodes)
 *   source         device; the nodal source values of step n (n = 0 .. steps-1,
 *                  i.e. at t_{n+1}) start at source + n * source_stride; a
 *                  stride of 0 reuses one vector; NULL = no source
 *   source_stride  >= 0, in elements
 * s (host, nullable) receives the statistics.  Returns the status, or a
 * negative error (wrong form, bad option).  Uses the handle's solver workspace;
 * synchronises the stream (one scalar readback per step). */
int egfem_burgers(egfem_tensor_t T, const uint8_t* dirichlet, const double* source, int64_t source_stride,
                  double* u, const egfem_burgers_opts* o, egfem_burgers_stats* s, void* stream);

/* ------------------------------------------------------------------------
 * Gradient nonlinearities with W_h = P0 (Sec. 3.2 gradient interpolation; the
 * p-Laplace and minimal surface examples of Sec. 5), solved like the paper by
 * Picard iteration:
 *     (T . a^n) u^{n+1} = d,   a^n_e = (c0 + c1 |grad u_h^n|_e|^2)^q  per cell e,
 * T the EGFEM_W_P0 tensor (T . a = sum_e a_e K^e), Dirichlet rows identity with
 * zero right-hand side.  p-Laplace: c0 = eps^2, c1 = 1, q = (p-2)/2; minimal
 * surface: c0 = c1 = 1, q = -1/2.  Each step: one cell kernel for a^n, the
 * emission of T . a^n (the A stream with the coefficient gathered per W-slot)
 * and one persistent preconditioned CG launch warm started from u^n.
 * ---------------------------------------------------------------------- */
typedef struct {
  double c0, c1, q;          /* a(z) = (c0 + c1 |z|^2)^q; c0, c1 >= 0 */
  int start_linear;          /* nonzero: the first step uses a = 1 (a Laplace solve), which also
                                starts p < 2 from u = 0 where a(0) is unbounded */
} egfem_grad_coef;

/* egfem_picard_grad: Picard iteration from u (device [n_nodes]; Dirichlet
 * entries set to 0) with the options of egfem_picard (tol on the relative
 * update, inexact CG relative to each step's initial residual).  p: load and
 * Dirichlet mask (a0 must be NULL, add_stiffness 0).  s->res receives ||F||
 * over the free rows at the returned iterate, F = T:(u (x) a(grad u)) - d (a
 * cell whose vertices are all Dirichlet nodes only couples Dirichlet nodes; its
 * coefficient may be unbounded without effect).  Returns the status or
 * EGFEM_ERR_ARG (not a W_h = P0 handle, bad parameters).  Synchronises. */
int egfem_picard_grad(egfem_tensor_t T, const egfem_problem* p, const egfem_grad_coef* g, double* u,
                      const egfem_picard_opts* o, egfem_picard_stats* s, void* stream);

/* egfem_newton_grad: damped Newton for the same problem (the rules of
 * egfem_newton: full steps halved while ||F|| does not fall by the factor
 * 1 - 1e-4 alpha, Eisenstat-Walker or fixed inner tolerance).  The Jacobian
 *     DF = T . a(grad u) + sum_e (K^e u_e) (x) (d a_e / d u),
 *     d a_e / d u_j = 2 q c1 (c0 + c1 |z_e|^2)^(q-1) z_e . grad lambda_j,
 * is symmetric; it is emitted by the W-slot stage with per-cell weights and
 * solved by preconditioned CG (BiCGStab if CG meets a non-positive curvature).  With
 * g->start_linear, u is first replaced by the Laplace solution (a = 1, CG to
 * 1e-12), the start from which s->res0 is measured; s->krylov_iters then
 * includes that solve's iterations, which s->krylov_hist (per Newton step)
 * does not hold.  Returns the status (EGFEM_STAGNATED as for egfem_newton) or
 * EGFEM_ERR_ARG.  Synchronises. */
int egfem_newton_grad(egfem_tensor_t T, const egfem_problem* p, const egfem_grad_coef* g, double* u,
                      const egfem_newton_opts* o, egfem_newton_stats* s, void* stream);

/* ------------------------------------------------------------------------
 * Launch shapes and the autotuner.
 * ---------------------------------------------------------------------- */
typedef struct {
  int action_runs;           /* workgroups of the tensor-action kernel, each over a contiguous
                                run of row blocks (0 = one workgroup per row block) */
  int action_pipe;           /* 1: software-pipelined runs (next block's stream loads issued
                                before the current block's gathers), 0: one block at a time */
  int krylov_blocks;         /* persistent Krylov grid (0 = default) */
  int krylov_threads;        /* persistent Krylov workgroup size 256/512/1024 (0 = default).  With
                                both 0 (an untuned handle): 256-thread workgroups with one row per
                                thread, ceil(n / 256) of them, where the register-resident kernel
                                applies and that grid is co-resident; else, in the Newton solver
                                (egfem_newton) of a handle with the block-Jacobi preconditioner,
                                1024-thread workgroups over the free rows (below) when they fit;
                                otherwise 1024 threads and min(ceil(n / 64), compute units)
                                workgroups of the streaming kernel */
  int krylov_kernel;         /* 0: register-resident BiCGStab (one thread per row) when every
                                workgroup's rows fit its threads, rows hold at most 8 entries
                                and workgroups have at most 512 threads, else the streaming
                                one.  Free rows: in egfem_newton the Dirichlet rows of the
                                Newton system are identity rows with zero residual, so with
                                1024-thread workgroups and the block-Jacobi preconditioner they
                                are left out (their correction is 0) and the barrier-form
                                resident BiCGStab runs one free row per thread on a compact
                                partition of the free rows (2D 512x512: 261,121 free rows on
                                256 workgroups, where 263,169 rows exceed the 256/512-thread
                                resident grids); the partition is rebuilt when the Dirichlet
                                mask's contents change.  The 1024-thread BiCGStab also runs
                                resident on every row where each part fits (linear solves,
                                systems without a mask).  3D meshes (rows of up to 16
                                entries) run only this form: 8 entries of a row in registers,
                                the others in the thread's slice of LDS.  egfem_adjoint leaves the
                                same rows out (DF^T keeps the identity rows and zero columns).
                                At 1024 threads the products read LDS: the part's own rows and
                                its ghosts (at most 1024, one coherent load per thread) are
                                staged there before each product (kernel 2: every column
                                gathered from memory).  With the block-Jacobi preconditioner the resident BiCGStab
                                runs in its overlapped form: every exchanged value (reduction
                                partials, gathered vector entries) carries its own completion
                                flag, the preconditioner's Chebyshev steps run while the
                                team's reductions complete, and in-part columns of a product
                                are read from LDS; 1: always the streaming one; 2: the resident
                                kernels in their barrier form (counter barriers, as the
                                streaming kernel) */
  int action_half;           /* 1: residual actions read the symmetric half stream (tensors with
                                T_ijk = T_ikj: mass, convection; each fiber keeps k at or after j,
                                the diagonal halved, and sums h a_k and h u_k), one row block per
                                workgroup; 0: the full stream (default; egfem_autotune picks the
                                half stream where it is faster) */
  int krylov_precond;        /* preconditioner of the register-resident BiCGStab: 0 = Jacobi
                                D^-1; k in 2..32 = block-Jacobi (default 8; 6 where rows hold more
                                than 8 entries, as on 3D meshes): the rows are split
                                by recursive coordinate bisection into one compact part per
                                workgroup, and each workgroup applies k Chebyshev steps (Jacobi
                                scaled, interval [lmax/ratio, lmax], ratio = krylov_cheb_ratio
                                (default 30), lmax the Gershgorin bound of
                                D^-1 J_b) to its diagonal block J_b: a fixed linear operator,
                                workgroup-local (LDS), with no synchronisation between
                                workgroups.  The register-resident CG uses the same operator
                                (symmetric positive definite for an SPD matrix: the polynomial
                                is positive on the spectrum); streaming kernels use Jacobi. */
  double krylov_cheb_ratio;  /* lmax / lmin of the Chebyshev interval of the block steps, in
                                [2, 1000]; 0 = 30 (the default) */
} egfem_launch_shape;

int egfem_get_shape(egfem_tensor_t T, egfem_launch_shape* s);
/* Set the shape used by later calls on this handle (e.g. restored from a
 * cache).  Out-of-range values give EGFEM_ERR_ARG. */
int egfem_set_shape(egfem_tensor_t T, const egfem_launch_shape* s);

/* Autotuner: time the candidate shapes on this handle's own tensor on
 * `stream` and keep the fastest in the handle.
 *   what: bit 0 -> tensor action (runs x {pipelined, not}, HIP events); bit 1 ->
 *         Krylov grid (kernel x threads x blocks, by the time of a damped Newton
 *         solve of problem p from u = 0 to 1e-10 with Eisenstat-Walker forcing,
 *         the second of two per candidate; p must then be non-NULL).
 *   best (host, nullable) receives the chosen shape; best_us (host [2], nullable)
 *   the chosen action launch time and, for the chosen grid, the Newton solve
 *   time per Krylov iteration in microseconds.
 * Overwrites the handle's solver workspace; allocates (and frees) one
 * temporary iterate.  Synchronises the stream. */
int egfem_autotune(egfem_tensor_t T, const egfem_problem* p, int what, egfem_launch_shape* best,
                   double* best_us, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint of the converged solve (implicit function theorem; the gradient
 * pattern for optimal control that motivates the method, Sec. 6).
 *
 * For an objective with dJ/du = ubar at the solution u* of F(u; d, a0) = 0:
 *   DF(u*)^T lambda = ubar on the free nodes (lambda = 0 on Dirichlet nodes),
 *   dJ/dd   = lambda                       (F depends on the load through -d),
 *   dJ/da0  = -(T ._2 u*)^T lambda, i.e. -sum_ij lambda_i T_ijk u*_j.
 * Only u* is needed (no Newton trajectory is stored).  The transposed
 * Jacobian is applied through the slot transpose permutation; the solve is the
 * same preconditioned BiCGStab with opts->krylov_rtol / max_krylov.
 *   u, ubar:      device [n_nodes] inputs
 *   lambda:       device [n_nodes] output (also dJ/dd)
 *   grad_a0:      device [n_nodes] output or NULL
 *   krylov_iters, relres: host outputs or NULL
 * Returns the Krylov status (EGFEM_OK / NOT_CONVERGED / BREAKDOWN / NONFINITE)
 * or a negative error.  Synchronises the stream.
 * ---------------------------------------------------------------------- */
int egfem_adjoint(egfem_tensor_t T, const egfem_problem* p, const double* u, const double* ubar,
                  const egfem_newton_opts* o, double* lambda, double* grad_a0, int* krylov_iters,
                  double* relres, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: `count` independent problems (each its own handle, sizes may
 * differ) solved by ONE persistent cooperative launch -- the many-query use the
 * paper's offline/online split is made for (Sec. 5 preamble).  Each instance
 * is owned by a team of workgroups sized by its tensor size; every team runs
 * the whole damped Newton loop (residual, Jacobian emission, BiCGStab, line
 * search, convergence test) on the device with team-local barriers, so there
 * is no host round trip.  us[m]: device [n_nodes of m], guess in / solution
 * out.  stats: host array [count] or NULL.  Same options for all instances
 * (timing is ignored).  Returns the worst instance status.  Synchronises.
 * ---------------------------------------------------------------------- */
int egfem_newton_batched(int count, const egfem_tensor_t* Ts, const egfem_problem* ps,
                         double* const* us, const egfem_newton_opts* o,
                         egfem_newton_stats* stats, void* stream);

/* Reusable batch plan behind egfem_newton_batched: device descriptors, team
 * assignment, control words and statistics buffers are built once; every run
 * is one persistent launch (plus a control-word fill and a statistics copy),
 * and egfem_batch_graph_run captures that sequence once in a hipGraph and
 * replays it.  The handles, problems and solution buffers passed at creation
 * must stay valid for the plan's life; a handle may appear only once in a
 * batch (its solver workspace is used by its team).
 *   threads:  workgroup size of the persistent kernel, 512 or 1024 (0 = 512)
 *   weight_exp: team share of instance m proportional to slots_m^weight_exp
 *             (0 = 1.5, the cost model iterations ~ n, work ~ n^2 per iteration)
 * Runs are asynchronous on `stream`; zero_init != 0 starts every instance from
 * u = 0 (else from the contents of its solution buffer). */
typedef struct egfem_batch_s* egfem_batch_t;
int egfem_batch_create(int count, const egfem_tensor_t* Ts, const egfem_problem* ps,
                       double* const* us, const egfem_newton_opts* o, int threads,
                       double weight_exp, egfem_batch_t* out);
/* Scheduled resident teams (the same run / graph / stats / destroy calls):
 * every team member owns at most `threads` consecutive rows (whole row
 * blocks), one per thread, so each Newton system is solved by the
 * register-resident BiCGStab with the block-Jacobi preconditioner of the
 * handle (krylov_precond Chebyshev steps on the member's rows; 0 = Jacobi).
 * The teams this needs exceed the co-resident workgroups, so the host packs
 * the instances into them in space and time: longest estimated duration
 * (n_nodes^dur_exp) first, each instance on the window of consecutive
 * workgroups that frees first; every workgroup then runs its (instance,
 * rank) list in start order within the one launch.  Requires rows of at
 * most 8 entries and W_h = P1 (EGFEM_ERR_ARG otherwise), and every team to
 * fit the resident workgroups (EGFEM_ERR_SHAPE otherwise).
 *   threads:  256 or 512 (0 = 256)
 *   dur_exp:  duration model exponent (0 = 0.5: Krylov iterations ~ h^-1) */
int egfem_batch_create_sched(int count, const egfem_tensor_t* Ts, const egfem_problem* ps,
                             double* const* us, const egfem_newton_opts* o, int threads,
                             double dur_exp, egfem_batch_t* out);
int egfem_batch_run(egfem_batch_t B, int zero_init, void* stream);
int egfem_batch_graph_run(egfem_batch_t B, int zero_init, void* stream);
/* Synchronises the stream and copies per-instance statistics into stats
 * (host array [count]); returns the worst status (largest code). */
int egfem_batch_stats(egfem_batch_t B, egfem_newton_stats* stats, void* stream);
/* Batch autotuner: time one eager run of the plan (the second of two, HIP
 * events on `stream`, every instance started from u = 0) for each candidate
 * -- streaming teams: workgroup size {512, 1024} x team weight exponent
 * {1, 1.5, 2}; scheduled resident teams (where they apply): workgroup size
 * {256, 512} x duration exponent {0.5, 1} -- on these instances and options,
 * and report the fastest whose instances all converge (EGFEM_OK, or
 * EGFEM_STAGNATED: stopped at the rounding floor of ||F||).  The solution
 * buffers are overwritten.  best_kind (0 streaming: egfem_batch_create, 1
 * scheduled: egfem_batch_create_sched), best_threads, best_exp (the weight or
 * duration exponent) and best_ms (host, nullable) receive the choice (the
 * Python binding caches it by the instance sizes).  EGFEM_ERR_ARG when no
 * candidate converges.  Synchronises the stream. */
int egfem_batch_autotune(int count, const egfem_tensor_t* Ts, const egfem_problem* ps,
                         double* const* us, const egfem_newton_opts* o, int* best_kind,
                         int* best_threads, double* best_exp, double* best_ms, void* stream);
/* Team size (workgroups) given to each instance: host array [count]; the
 * workgroups of the launch. */
int egfem_batch_teams(egfem_batch_t B, int* team_sizes, int* total_workgroups);
void egfem_batch_destroy(egfem_batch_t B);

/* ------------------------------------------------------------------------
 * Measurement aid: the streaming-read ceiling.  A plain read of x with the
 * tensor action's launch arrangement (one contiguous chunk of
 * egfem_stream_read_chunks granularity per workgroup, every 16-byte load of a
 * thread issued before the first is used, chunks mapped to the XCDs in
 * contiguous regions); the bandwidth it reaches on a buffer that is not in
 * the caches is the measured reference for the tensor action's HBM fraction.
 *   x        device [n] doubles (16-byte aligned for the vector path)
 *   partial  device [n_partial] doubles, n_partial >= egfem_stream_read_chunks(n);
 *            partial[c] receives the sum of chunk c (2048 doubles, the last
 *            one shorter)
 * Asynchronous on `stream`.  EGFEM_ERR_ARG for null pointers or n < 0,
 * EGFEM_ERR_SHAPE when partial is too short.
 * ---------------------------------------------------------------------- */
int64_t egfem_stream_read_chunks(int64_t n);
int egfem_stream_read(const double* x, int64_t n, double* partial, int64_t n_partial, void* stream);

/* Thread-local message of the last error. */
const char* egfem_last_error(void);

/* Library version string. */
const char* egfem_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EGFEM_H */
