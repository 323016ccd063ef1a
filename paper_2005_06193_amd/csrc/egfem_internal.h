// Internal declarations shared by the libegfem translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/egfem.h"

namespace egfem {

// Row-block capacities of the LDS-staged tensor kernels.  A block is a run of
// consecutive node rows whose A-stream entries, B-stream entries and
// adjacency slots all fit these bounds (one workgroup per block).
constexpr int kBlockThreads = 256;
constexpr int kCapNnz = 1024;     // tensor entries per block (A and B separately)
constexpr int kCapSlots = 512;    // adjacency slots per block
constexpr int kCapRows = 256;     // rows per block (one thread per row in the row stage)
constexpr int kCapWSlots = 1024;  // W-slots per block (W_h = P2: P2 dofs coupled to the block's rows)

// Persistent Krylov kernel shape.
constexpr int kKrylovThreads = 1024;
constexpr int kMaxKrylovBlocks = 1024;
constexpr int kResidentRow = 8;    // most entries of a row in the register-resident Krylov forms
constexpr int kWideRow = 8;        // entries past those the 1024-thread resident BiCGStab keeps in LDS
constexpr int kRedSlots = 10;     // reduction slots in flight (>= 2 barriers apart)
constexpr int kCtrlWordsMax = 4096;  // barrier control words and publication flags
constexpr int kMaxNbrLists = 16;     // neighbour workgroups kept per workgroup (more, for any
                                     // workgroup: every workgroup uses the team barrier)

// Compact row partition of the register-resident Krylov solvers (recursive
// coordinate bisection into G parts of balanced size).
struct CompactPartition {
  std::vector<int32_t> kr;      // [G+1] part offsets into rlist
  std::vector<int32_t> rlist;   // [n] rows of every part, ascending within a part
  std::vector<int16_t> kloc;    // [slots] row-local position of the column in the row's part, or -1
  std::vector<int32_t> nbr;     // [G][kMaxNbrLists + 1] neighbour lists (count or -1, parts)
  int maxrows = 0;
};
// skip (host, nullable): rows marked nonzero are left out of every part (the
// Dirichlet rows of a Newton system: identity rows with zero right-hand side).
int make_compact_partition(int dim, const double* X, int64_t n, const int32_t* rowptr, const int32_t* col, int G,
                           CompactPartition& out, const uint8_t* skip = nullptr);
// Neighbour lists [G][kMaxNbrLists + 1]: when any workgroup's list overflowed
// (count -1), mark every list -1 (all workgroups then take the team barrier).
void uniform_neighbor_lists(std::vector<int32_t>& nbr, int G);

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define EGFEM_HIP_CHECK(expr)                                                        \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::egfem::fail(EGFEM_ERR_HIP, std::string(#expr " failed: ") +          \
                                              hipGetErrorString(e_));                \
  } while (0)

// A Krylov launch whose outcome has not been read yet.
struct KrylovPending {
  bool active = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // launch timing (timed solves)
  int G = 0, NT = 0;
  bool resident = false, block = false, overlapped = false;
};

// Solver workspace owned by a handle (allocated on first use).
struct Workspace {
  bool ready = false;
  double* F = nullptr;          // residual
  double* delta = nullptr;      // Newton correction
  double* utry = nullptr;       // damped trial iterate
  double* jval = nullptr;       // Jacobian values [slots]
  double* jvalT = nullptr;      // transposed values [slots] (adjoint solves)
  double* dinv = nullptr;       // 1 / diag
  double* rhs = nullptr;
  // BiCGStab vectors
  double *r = nullptr, *rhat = nullptr, *p = nullptr, *v = nullptr, *s = nullptr,
         *t = nullptr, *z = nullptr, *phat = nullptr, *rh = nullptr, *vh = nullptr;
  double* partial = nullptr;    // per-workgroup partial sums of the action kernel [row_blocks]
  double* red = nullptr;        // persistent-kernel reduction slots [kRedSlots * 8 * kMaxKrylovBlocks]
  unsigned* ctrl = nullptr;     // barrier counters / epoch / abort flag [kCtrlWordsMax] (device)
  // free-row partition (rows left out of the resident solve): the mask it was
  // built for (host copy) and its device pointer
  std::vector<uint8_t> crow_skip;
  const uint8_t* crow_skip_dev = nullptr;
  bool crow_free = false;       // the compact partition in crow/crlist leaves those rows out
  double* qslot = nullptr;      // per-slot scratch [qslot_len >= slots] (mode-3 contraction,
                                //   f on the dofs of W_h in the Burgers group steps)
  int64_t qslot_len = 0;
  int32_t* krow = nullptr;      // Krylov row partition [kMaxKrylovBlocks + 1]
  int krow_blocks = 0;          // grid size the partition was made for
  int krow_maxrows = 0;         // most rows of one workgroup in that partition
  int32_t* knbr = nullptr;      // per workgroup: neighbour count (-1: too many), ranks
  // compact partition of the block-Jacobi preconditioner (recursive coordinate bisection)
  int32_t* crow = nullptr;      // [kMaxKrylovBlocks + 1] part offsets into crlist
  int32_t* crlist = nullptr;    // [n] rows of every part
  int16_t* ckloc = nullptr;     // [slots] row-local column position within the part, or -1
  int32_t* cnbr = nullptr;      // neighbour lists of the parts
  int crow_blocks = 0;          // grid size the compact partition was made for
  int crow_maxrows = 0;
  int crow_maxghost = 0;        // most ghost columns (out-of-part columns of its rows) of a part
  int16_t* ckext = nullptr;     // [slots] LDS position of the column: part-local, or -1 - ghost index
  int32_t* cgptr = nullptr;     // [kMaxKrylovBlocks + 1] ghost range of every part
  int32_t* cgcol = nullptr;     // [slots] global column of every ghost
  // flagged exchange of the overlapped block-Jacobi BiCGStab
  uint64_t* llv = nullptr;      // flagged words: [3][n][2] published vectors, then the reduction words
  unsigned ll_salt = 0;         // 1 .. 4095, advanced at every launch (0: buffer not yet zeroed)
  double* kout = nullptr;       // Krylov result [4] (device)
  double* host_partial = nullptr;  // pinned host mirror of partial sums
  double* host_kout = nullptr;     // pinned host mirror of the Krylov result
  std::vector<hipEvent_t> timer_events;   // events of the drivers' launch timing (reused)
  KrylovPending kpend;                    // the Krylov launch in flight (deferred collection)
};

}  // namespace egfem

// The handle.
struct egfem_tensor_s {
  int dim = 0;
  int form = 0;
  int symmetric = 0;
  int64_t n = 0;
  int64_t n_cells = 0;
  int64_t nnz = 0;
  int64_t nnz_b = 0;
  int64_t structural = 0;
  int64_t slots = 0;
  int max_row_slots = 0;
  int lanes_per_row = 8;        // SpMV sub-wave width (power of two >= max row length)
  int krylov_lanes = 4;         // persistent-Krylov SpMV width (power of two >= max row / 2)
  int krylov_rs = 4;            // streaming-Krylov row shape code (see row_L / row_K)
  int action_runs_target = 0;   // workgroups of the action kernel (block runs; 0 = one per block)
  int action_pipe = 0;          // 1: software-pipelined block runs
  int tuned_krylov_blocks = 0;  // Krylov grid chosen by the autotuner (0 = heuristic)
  int tuned_krylov_threads = 0;
  int krylov_kernel = 0;        // 0: register-resident where it fits, 1: streaming
  int krylov_precond = 8;       // 0: Jacobi; k >= 2: block-Jacobi, k Chebyshev steps per block (resident BiCGStab)
  double krylov_cheb_ratio = 30.0;   // Chebyshev interval [lmax / ratio, lmax] of the block steps
  int device = 0;
  // W_h = P2 (Case 1, w2 = 1): k runs over the P2 dofs (vertices, then edges);
  // W_h = I_k (Case 3, w2 = 2): k runs over the quadrature points of the cells;
  // W_h = P0 (w2 = 3): k runs over the cells (gradient nonlinearities)
  int w2 = 0;
  int nq = 0;                   // I_k: points per cell
  int64_t n_w = 0;              // dofs of W_h (n for P1)
  int64_t wslots = 0;           // W-slots: (row, P2 dof) couplings
  int max_row_wslots = 0;
  // device arrays
  int32_t* rowptr = nullptr;    // [n+1]
  int32_t* col = nullptr;       // [slots]
  int32_t* diag = nullptr;      // [n]   slot of (i,i)
  int32_t* tperm = nullptr;     // [slots] slot of (j,i) for slot (i,j)
  int32_t* kptrA = nullptr;     // [slots+1]
  int32_t* kA = nullptr;        // [nnz]
  double* vA = nullptr;         // [nnz]
  int32_t* jptrB = nullptr;     // [slots+1]  (aliases kptrA when symmetric)
  int32_t* jB = nullptr;        // [nnz]
  double* vB = nullptr;         // [nnz]
  uint16_t* kS = nullptr;       // [nnz]  block-relative slot of (i, k) of every A entry
  uint16_t* bS = nullptr;       // [nnz]  block-relative B position of every A entry (not symmetric)
  uint16_t* kpS = nullptr;      // [slots] A fiber start relative to the block's first A entry
  uint16_t* jpS = nullptr;      // [slots] B fiber start relative to the block's first B entry (aliases)
  double* kval = nullptr;       // [slots]
  double* mval = nullptr;       // [slots]
  int32_t* blk_row = nullptr;   // [row_blocks+1]
  int32_t* blk_meta = nullptr;  // [row_blocks*8]: rows, slots, A range, B range of each block
  int32_t* wrowptr = nullptr;   // W_h = P2: [n+1] W-slot range of every row
  int32_t* wcol = nullptr;      //   [wslots] P2 dof of every W-slot
  uint32_t* wpq = nullptr;      //   [wslots] block-relative slots of its endpoints, p | q << 16
  int32_t* wmeta = nullptr;     //   [row_blocks*2] W-slot range of every block
  // symmetric half stream (T_ijk = T_ikj): residual actions may use it
  int64_t nnz_h = 0;
  int action_half = 0;          // 1: residual actions read the half stream
  uint16_t* kSH = nullptr;      // [nnz_h] block-relative slot of (i, k), k at or after j
  double* vH = nullptr;         // [nnz_h] values, diagonal entries halved
  uint16_t* kpSH = nullptr;     // [slots] half fiber start relative to the block's first half entry
  int32_t* hmeta = nullptr;     // [row_blocks*2] half-stream range of every block
  // element-factored form of the stiffness tensor (optional)
  int64_t e_cells = 0;
  int e_kstride = 0;            // doubles per packed K^e (triangle of (d+1)^2, rounded to even)
  int e_lanes = 0;              // lanes per row of the element action (power of two >= max incidence)
  int4* e_cell4 = nullptr;      // [cells] vertex ids, padded with the first
  double* e_kp = nullptr;       // [cells * kstride] packed K^e (row-major upper triangle)
  int32_t* e_nptr = nullptr;    // [n+1] incidence range of every node
  int32_t* e_inc = nullptr;     // [incidences] cell << 2 | local index
  double* e_grad = nullptr;     // W_h = P0: [cells * 12] grad lambda_m of every cell (4 x 3, padded)
  double* e_acoef = nullptr;    // W_h = P0: [cells] coefficient buffer of egfem_picard_grad / egfem_newton_grad
  double* e_wv = nullptr;       // W_h = P0: [cells * 4] derivative weights of the Newton Jacobian
  int32_t* p2_edges = nullptr;  // W_h = P2: [edges * 2] endpoints of every edge dof
  // unique storage of the fully symmetric mass tensor (optional): every index
  // multiset {i,j,k} once, as T_iii, then per edge (a < b) T_aab, T_abb, then per face T_abc
  int64_t u_count = 0;          // N + 2E + F stored values
  int64_t u_foff = 0;           // N + 2E: first face value
  int u_lanes = 0;              // lanes per row of the unique-storage action
  int u_stride = 0;             // LDS entries per row (most slots of a row)
  double* u_val = nullptr;      // [u_count]
  int32_t* u_sref = nullptr;    // [slots] 2 e + (i > j) for slot (i, j), j != i
  int32_t* u_fptr = nullptr;    // [n+1] face-reference range of every row
  int2* u_fref = nullptr;       // [3F] (face id, row-local slots of the other two vertices s_j | s_k << 16)
  uint32_t* wpq2 = nullptr;     // I_k: [wslots] slots of the third and fourth cell vertex
  uint8_t* wqi = nullptr;       // I_k: [wslots] point index
  double* qlam = nullptr;       // I_k: [4*4] barycentrics of the points
  int64_t row_blocks = 0;
  std::vector<int32_t> h_rowptr;  // host copy (row partitions)
  std::vector<int32_t> h_col;     // host copy (neighbour lists of a partition)
  std::vector<double> h_coords;   // host copy of the node coordinates (compact partitions)
  int64_t device_bytes = 0;
  egfem::Workspace ws;
};

namespace egfem {

// Row shapes of the streaming BiCGStab SpMV, by code: L lanes per row, K
// entries per lane loaded at once (rows of up to L*K entries need no tail loop).
constexpr int kRowShapes = 9;
constexpr int kRowShapeLK[kRowShapes][2] = {{1, 8}, {2, 4}, {4, 2}, {8, 2}, {16, 2},
                                            {32, 2}, {64, 2}, {1, 16}, {2, 8}};
constexpr int row_L(int rs) { return kRowShapeLK[rs][0]; }
constexpr int row_K(int rs) { return kRowShapeLK[rs][1]; }
// Shape for rows of at most max_row_slots entries (lanes: power of two >= max_row / 2).
inline int row_shape_for(int max_row_slots, int lanes) {
  if (max_row_slots <= 8) return 0;     // (1, 8): one thread per row
  if (max_row_slots <= 16) return 8;    // (2, 8)
  switch (lanes) {
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
    case 32: return 5;
    default: return 6;
  }
}

// Kernel launchers (egfem_kernels.hip).  All return hipError_t of the launch.
struct ProblemView {
  const double* a0;       // or null
  double a0c;
  const double* load;     // or null (treated as 0)
  const uint8_t* dir;     // or null
  int addK;
};

int64_t action_runs(const egfem_tensor_s* T);
hipError_t launch_action_raw(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                             hipStream_t st);
// a_e = (c0 + c1 |grad u_h|_e|^2)^q over the cells of a W_h = P0 handle (linear: a_e = 1).
hipError_t launch_grad_coef(const egfem_tensor_s* T, const double* u, double c0, double c1, double q, int linear,
                            double* a, double* wv, hipStream_t st);
// Newton Jacobian of a gradient nonlinearity (W_h = P0): T . a plus the
// per-cell derivative weights wv [4 per cell] applied to (K^e u)_i.
hipError_t launch_jacobian_grad(const egfem_tensor_s* T, const double* a, const double* u, const double* wv,
                                const uint8_t* dir, double* jval, double* dinv, hipStream_t st);
// F = mask(F - b) with partial sums of F^2 into partial[g] (returns the workgroup count, at most 256).
int launch_sub_mask_norm(int64_t n, double* F, const double* b, const uint8_t* dir, double* partial, hipStream_t st,
                         hipError_t* err);
hipError_t launch_axpy(double* out, const double* x, double alpha, const double* y, int64_t n, hipStream_t st);
// f = (Pi_u u)^2 at the P2 dofs: u_k^2 at the vertices, ((u_x + u_y) / 2)^2 at the edges.
hipError_t launch_p2_square(const egfem_tensor_s* T, const double* u, double* f, hipStream_t st);
hipError_t launch_iq_square(const egfem_tensor_s* T, const double* u, double* f, hipStream_t st);
hipError_t launch_action_elementwise(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                                     hipStream_t st);
hipError_t launch_action_unique(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                                hipStream_t st);
hipError_t launch_action_problem(const egfem_tensor_s* T, const ProblemView& pv, const double* u,
                                 const double* delta, double alpha, double* uout, double* F,
                                 double* partial, hipStream_t st);
hipError_t launch_jacobian(const egfem_tensor_s* T, const double* u, const double* a,
                           const double* a0, double a0c, int use_problem_a, const double* dadu,
                           int dadu_2u, int addK, const uint8_t* dir, double* jval, double* dinv,
                           hipStream_t st);
hipError_t launch_slot_mode2(const egfem_tensor_s* T, const double* u, double* q, hipStream_t st);
// Partial sums of (x - u)^2 and x^2 into partial[2 g], partial[2 g + 1] for
// the returned number of workgroups g (at most 256).
int launch_diff_norms(int64_t n, const double* x, const double* u, double* partial, hipStream_t st,
                      hipError_t* err);
hipError_t launch_csr_matvec(const egfem_tensor_s* T, const double* vals, const double* x, double* y,
                             hipStream_t st);
hipError_t launch_csr_matvec_perm(const egfem_tensor_s* T, const double* vals, const double* w,
                                  double* y, hipStream_t st);
hipError_t launch_permute_slots(const egfem_tensor_s* T, const double* in, double* out,
                                hipStream_t st);
// vals = cm M + ck K in T's pattern with Dirichlet identity rows and zero
// columns; dinv = 1 / diagonal.
hipError_t launch_mk_combine(const egfem_tensor_s* T, double cm, double ck, const uint8_t* dir, double* vals,
                             double* dinv, hipStream_t st);
// u <- extrapolation of order 0..2 from u, h1, h2; then h2 <- h1, h1 <- old u.
hipError_t launch_extrapolate(int64_t n, int order, double* u, double* h1, double* h2, hipStream_t st);
// Burgers right-hand side M (u + dt src) + dt/2 C; cvals = N^f in slot layout
// (group) or the tensor action N:(u (x) u) [n] (tensor formulation).
hipError_t launch_burgers_rhs(const egfem_tensor_s* T, bool group, const double* u, const double* src, double dt,
                              const double* cvals, const uint8_t* dir, double* rhs, hipStream_t st);
hipError_t launch_fill(double* x, double v, int64_t n, hipStream_t st);
hipError_t launch_fill_u32(unsigned* x, unsigned v, int64_t n, hipStream_t st);
hipError_t launch_mask_zero(double* x, const uint8_t* dir, int64_t n, hipStream_t st);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t st);
hipError_t launch_scale(double* x, double s, int64_t n, hipStream_t st);

// Krylov (egfem_krylov.hip)
struct KrylovResult {
  int status = 0;
  int iters = 0;
  double relres = 0.0;
  double bnorm = 0.0;
  int blocks = 0;
  int threads = 0;
  double kernel_ms = 0.0;   // launch duration of the persistent kernel (when timed)
  bool resident = false;    // the register-resident kernel ran
  bool block_precond = false;   // with the block-Jacobi preconditioner
  bool overlapped = false;      // the overlapped (flagged-synchronisation) BiCGStab ran
};
enum class KrylovMethod { kBiCGStab, kCG };

// Persistent preconditioned Krylov solve of (rhs_scale * rhs) = A x,
// A = J (perm == null) or J^T (perm = tperm); conjugate gradients need an SPD
// J.  Stops when ||r|| <= rtol ||b|| (or rtol ||r0|| with rel_r0).  With
// defer, the call returns once the launch and the copy of its outcome are
// enqueued; krylov_collect synchronises the stream and fills res (one solve
// in flight per handle).
int krylov_solve(KrylovMethod method, egfem_tensor_s* T, const double* jval, const double* dinv,
                 const double* rhs, double rhs_scale, double* x, bool x_zero, double rtol, bool rel_r0,
                 int max_iter, int blocks, KrylovResult* res, hipStream_t st, const int32_t* perm,
                 bool timed = false, int threads = 0, bool defer = false, const uint8_t* skip_rows = nullptr);
int krylov_collect(egfem_tensor_s* T, hipStream_t st, KrylovResult* res);
inline int krylov_bicgstab(egfem_tensor_s* T, const double* jval, const double* dinv, const double* rhs,
                           double rhs_scale, double* x, bool x_zero, double rtol, int max_iter, int blocks,
                           KrylovResult* res, hipStream_t st, const int32_t* perm, bool timed = false,
                           int threads = 0, bool defer = false, const uint8_t* skip_rows = nullptr) {
  return krylov_solve(KrylovMethod::kBiCGStab, T, jval, dinv, rhs, rhs_scale, x, x_zero, rtol, false, max_iter,
                      blocks, res, st, perm, timed, threads, defer, skip_rows);
}

// Workspace
int ensure_workspace(egfem_tensor_s* T);

}  // namespace egfem
