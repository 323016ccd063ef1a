// C entry points of libegfem: handle lifecycle, tensor actions, the Newton
// driver (Sec. 4) and the Jacobi-BiCGStab solve.  Argument checks happen here;
// the device work is in egfem_kernels.hip and egfem_krylov.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "egfem_internal.h"

namespace egfem {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename T>
static int dalloc(T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return fail(EGFEM_ERR_OOM, "hipMalloc of solver workspace failed");
  return EGFEM_OK;
}

int ensure_workspace(egfem_tensor_s* T) {
  Workspace& W = T->ws;
  if (W.ready) return EGFEM_OK;
  const size_t N = (size_t)T->n, S = (size_t)T->slots;
  int rc = EGFEM_OK;
  double** nvecs[] = {&W.F, &W.delta, &W.utry, &W.dinv, &W.rhs, &W.r, &W.rhat, &W.p,
                      &W.v, &W.s, &W.t, &W.z, &W.phat, &W.rh, &W.vh};
  for (double** v : nvecs)
    if (rc == EGFEM_OK) rc = dalloc(v, N);
  if (rc == EGFEM_OK) rc = dalloc(&W.jval, S);
  if (rc == EGFEM_OK) rc = dalloc(&W.jvalT, S);
  // the Burgers group steps with W_h = P2 or I_k stage f on the n_w dofs here
  const size_t QS = (T->w2 == 1 || T->w2 == 2) ? std::max(S, (size_t)T->n_w) : S;
  if (rc == EGFEM_OK) rc = dalloc(&W.qslot, QS);
  W.qslot_len = (int64_t)QS;
  if (rc == EGFEM_OK) rc = dalloc(&W.partial, (size_t)T->row_blocks);
  if (rc == EGFEM_OK) rc = dalloc(&W.red, (size_t)kRedSlots * 8 * kMaxKrylovBlocks);
  if (rc == EGFEM_OK) rc = dalloc(&W.ctrl, kCtrlWordsMax);
  if (rc == EGFEM_OK) rc = dalloc(&W.krow, (size_t)kMaxKrylovBlocks + 1);
  if (rc == EGFEM_OK) rc = dalloc(&W.knbr, (size_t)kMaxKrylovBlocks * (kMaxNbrLists + 1));
  if (rc == EGFEM_OK) rc = dalloc(&W.kout, 4);
  if (rc == EGFEM_OK &&
      hipHostMalloc((void**)&W.host_partial, std::max<size_t>(T->row_blocks, 1) * sizeof(double), 0) != hipSuccess)
    rc = fail(EGFEM_ERR_OOM, "hipHostMalloc failed");
  if (rc == EGFEM_OK && hipHostMalloc((void**)&W.host_kout, 4 * sizeof(double), 0) != hipSuccess)
    rc = fail(EGFEM_ERR_OOM, "hipHostMalloc failed");
  if (rc != EGFEM_OK) return rc;
  T->device_bytes += (int64_t)((15 * N + 2 * S + QS + T->row_blocks + (size_t)kRedSlots * 8 * kMaxKrylovBlocks + 4) *
                                   sizeof(double) + (kMaxKrylovBlocks + 1) * 4 + kCtrlWordsMax * 4 +
                               (int64_t)kMaxKrylovBlocks * (kMaxNbrLists + 1) * 4);
  W.krow_blocks = 0;
  W.ready = true;
  return EGFEM_OK;
}

static void free_workspace(Workspace& W) {
  double* vecs[] = {W.F,  W.delta, W.utry, W.jval, W.jvalT, W.dinv, W.rhs,     W.r,
                    W.rhat, W.p,  W.v,     W.s,    W.t,    W.z,    W.phat,  W.rh,
                    W.vh, W.partial, W.red, W.qslot, W.kout};
  for (double* v : vecs)
    if (v) hipFree(v);
  if (W.ctrl) hipFree(W.ctrl);
  if (W.krow) hipFree(W.krow);
  if (W.knbr) hipFree(W.knbr);
  if (W.crow) hipFree(W.crow);
  if (W.cnbr) hipFree(W.cnbr);
  if (W.crlist) hipFree(W.crlist);
  if (W.ckloc) hipFree(W.ckloc);
  if (W.llv) hipFree(W.llv);
  if (W.ckext) hipFree(W.ckext);
  if (W.cgptr) hipFree(W.cgptr);
  if (W.cgcol) hipFree(W.cgcol);
  if (W.host_partial) hipHostFree(W.host_partial);
  if (W.host_kout) hipHostFree(W.host_kout);
  if (W.kpend.ev0) hipEventDestroy(W.kpend.ev0);
  if (W.kpend.ev1) hipEventDestroy(W.kpend.ev1);
  for (hipEvent_t e : W.timer_events) hipEventDestroy(e);
  W = Workspace();
}

__global__ void k_diag_inv(int64_t n, const int32_t* __restrict__ diag, const double* __restrict__ jval,
                           double* __restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dinv[i] = 1.0 / jval[diag[i]];
}

// ||F||_2 from the per-block partial sums written by the fused residual kernel,
// added on the host in block order (deterministic).
static int read_norm(egfem_tensor_s* T, hipStream_t st, double* norm) {
  Workspace& W = T->ws;
  const int64_t nrun = action_runs(T);
  EGFEM_HIP_CHECK(hipMemcpyAsync(W.host_partial, W.partial, nrun * sizeof(double), hipMemcpyDeviceToHost, st));
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  double s = 0.0;
  for (int64_t b = 0; b < nrun; ++b) s += W.host_partial[b];
  *norm = std::sqrt(s);
  return EGFEM_OK;
}

// Launch-duration accounting with HIP events on the caller's stream: every
// start/stop pair records two events; the durations are read once, at
// finish(), after the last event completes, so timing adds no host
// synchronisation inside a solve.
struct LaunchTimer {
  struct Pending {
    hipEvent_t a, b;
    double* acc;
    int* cnt;
  };
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t>* pool = nullptr;   // the handle's events, reused from call to call
  size_t used = 0;
  std::vector<Pending> pending;
  hipEvent_t cur = nullptr;
  int init(bool enable, hipStream_t s, std::vector<hipEvent_t>* events) {
    on = enable;
    st = s;
    pool = events;
    return EGFEM_OK;
  }
  int record(hipEvent_t* e) {
    if (used == pool->size()) {
      hipEvent_t ne = nullptr;
      EGFEM_HIP_CHECK(hipEventCreate(&ne));
      pool->push_back(ne);
    }
    *e = (*pool)[used++];
    EGFEM_HIP_CHECK(hipEventRecord(*e, st));
    return EGFEM_OK;
  }
  int start() {
    if (!on) return EGFEM_OK;
    return record(&cur);
  }
  int stop(double* acc, int* cnt) {
    if (!on) return EGFEM_OK;
    hipEvent_t b = nullptr;
    const int rc = record(&b);
    if (rc != EGFEM_OK) return rc;
    pending.push_back({cur, b, acc, cnt});
    return EGFEM_OK;
  }
  // Add the recorded durations to their accumulators.
  int finish() {
    if (!on || pending.empty()) return EGFEM_OK;
    EGFEM_HIP_CHECK(hipEventSynchronize(pending.back().b));
    for (const Pending& q : pending) {
      float ms = 0.0f;
      EGFEM_HIP_CHECK(hipEventElapsedTime(&ms, q.a, q.b));
      *q.acc += ms;
      ++*q.cnt;
    }
    pending.clear();
    used = 0;
    return EGFEM_OK;
  }
};

#define EGFEM_TRY_RC(x)                    \
  do {                                     \
    if ((rc = (x)) != EGFEM_OK) return rc; \
  } while (0)

static ProblemView view(const egfem_problem* p) {
  ProblemView v;
  v.a0 = p->a0;
  v.a0c = p->a0_const;
  v.load = p->load;
  v.dir = p->dirichlet;
  v.addK = p->add_stiffness;
  return v;
}

}  // namespace egfem

using namespace egfem;

extern "C" {

const char* egfem_last_error(void) { return g_last_error.c_str(); }

const char* egfem_version(void) { return "egfem-gfx950 0.1"; }

void egfem_tensor_destroy(egfem_tensor_t T) {
  if (!T) return;
  free_workspace(T->ws);
  void* ptrs[] = {T->rowptr, T->col,  T->diag,    T->tperm,    T->kptrA, T->kA,   T->vA,   T->kS,
                  T->kpS,    T->kval, T->mval,    T->blk_row,  T->blk_meta, T->wrowptr, T->wcol, T->wpq,
                  T->wmeta,  T->wpq2, T->wqi,       T->qlam,   T->e_cell4, T->e_kp,    T->e_nptr,
                  T->e_inc,  T->kSH,  T->vH,        T->kpSH,   T->hmeta,   T->e_grad,  T->e_acoef,
                  T->e_wv,   T->p2_edges, T->u_val,   T->u_sref,  T->u_fptr,  T->u_fref};
  for (void* p : ptrs)
    if (p) hipFree(p);
  if (!T->symmetric) {
    if (T->jptrB) hipFree(T->jptrB);
    if (T->jB) hipFree(T->jB);
    if (T->vB) hipFree(T->vB);
    if (T->bS) hipFree(T->bS);
    if (T->jpS) hipFree(T->jpS);
  }
  delete T;
}

int egfem_tensor_info(egfem_tensor_t T, egfem_info* info) {
  if (!T || !info) return fail(EGFEM_ERR_ARG, "null argument");
  info->dim = T->dim;
  info->form = T->form;
  info->symmetric = T->symmetric;
  info->n_nodes = T->n;
  info->n_cells = T->n_cells;
  info->nnz = T->nnz;
  info->nnz_b = T->nnz_b;
  info->structural_nnz = T->structural;
  info->slots = T->slots;
  info->row_blocks = T->row_blocks;
  info->device_bytes = T->device_bytes;
  info->rowptr = T->rowptr;
  info->col = T->col;
  info->kval = T->kval;
  info->mval = T->mval;
  info->wspace = T->w2;   // EGFEM_W_P1 / EGFEM_W_P2 / EGFEM_W_IQ
  info->n_w = T->n_w;
  info->nnz_half = T->nnz_h;
  return EGFEM_OK;
}

int egfem_tensor_export(egfem_tensor_t T, int32_t* i, int32_t* j, int32_t* k, double* v) {
  if (!T || !i || !j || !k || !v) return fail(EGFEM_ERR_ARG, "null argument");
  std::vector<int32_t> kptr(T->slots + 1), col(T->slots);
  EGFEM_HIP_CHECK(hipMemcpy(kptr.data(), T->kptrA, kptr.size() * 4, hipMemcpyDeviceToHost));
  EGFEM_HIP_CHECK(hipMemcpy(col.data(), T->col, col.size() * 4, hipMemcpyDeviceToHost));
  EGFEM_HIP_CHECK(hipMemcpy(k, T->kA, T->nnz * 4, hipMemcpyDeviceToHost));
  EGFEM_HIP_CHECK(hipMemcpy(v, T->vA, T->nnz * 8, hipMemcpyDeviceToHost));
  for (int64_t r = 0; r < T->n; ++r)
    for (int32_t s = T->h_rowptr[r]; s < T->h_rowptr[r + 1]; ++s)
      for (int32_t p = kptr[s]; p < kptr[s + 1]; ++p) {
        i[p] = (int32_t)r;
        j[p] = col[s];
      }
  return EGFEM_OK;
}

int egfem_tensor_pattern(egfem_tensor_t T, int32_t* rowptr, int32_t* col) {
  if (!T || !rowptr || !col) return fail(EGFEM_ERR_ARG, "null argument");
  std::memcpy(rowptr, T->h_rowptr.data(), (T->n + 1) * sizeof(int32_t));
  EGFEM_HIP_CHECK(hipMemcpy(col, T->col, T->slots * sizeof(int32_t), hipMemcpyDeviceToHost));
  return EGFEM_OK;
}

int egfem_residual(egfem_tensor_t T, const double* u, const double* a, double* r, void* stream) {
  if (!T || !u || !a || !r) return fail(EGFEM_ERR_ARG, "null argument");
  if (r == u || r == a) return fail(EGFEM_ERR_ARG, "r must not alias u or a");
  EGFEM_HIP_CHECK(launch_action_raw(T, u, a, r, (hipStream_t)stream));
  return EGFEM_OK;
}

int egfem_residual_elementwise(egfem_tensor_t T, const double* u, const double* a, double* r, void* stream) {
  if (!T || !u || !a || !r) return fail(EGFEM_ERR_ARG, "null argument");
  if (!T->e_kp) return fail(EGFEM_ERR_ARG, "no element data attached (egfem_attach_elements)");
  if (r == u || r == a) return fail(EGFEM_ERR_ARG, "r must not alias u or a");
  EGFEM_HIP_CHECK(launch_action_elementwise(T, u, a, r, (hipStream_t)stream));
  return EGFEM_OK;
}

int egfem_residual_unique(egfem_tensor_t T, const double* u, const double* a, double* r, void* stream) {
  if (!T || !u || !a || !r) return fail(EGFEM_ERR_ARG, "null argument");
  if (!T->u_val) return fail(EGFEM_ERR_ARG, "no unique storage attached (egfem_attach_unique)");
  if (r == u || r == a) return fail(EGFEM_ERR_ARG, "r must not alias u or a");
  EGFEM_HIP_CHECK(launch_action_unique(T, u, a, r, (hipStream_t)stream));
  return EGFEM_OK;
}

int egfem_jacobian(egfem_tensor_t T, const double* u, const double* a, const double* dadu,
                   int add_stiffness, const uint8_t* dirichlet, double* jval, double* dinv,
                   void* stream) {
  if (!T || !u || !a || !jval) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3 && dadu) return fail(EGFEM_ERR_ARG, "W_h = P0 handles emit the first Jacobian term only");
  EGFEM_HIP_CHECK(launch_jacobian(T, u, a, nullptr, 0.0, 0, dadu, 0, add_stiffness, dirichlet, jval,
                                  dinv, (hipStream_t)stream));
  return EGFEM_OK;
}

int egfem_mode3(egfem_tensor_t T, const double* w, const double* u, double* out, void* stream) {
  if (!T || !w || !u || !out) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2) return fail(EGFEM_ERR_ARG, "mode-3 contraction is not available for handles with W_h != P1");
  if (out == w || out == u) return fail(EGFEM_ERR_ARG, "out must not alias w or u");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  EGFEM_HIP_CHECK(launch_slot_mode2(T, u, T->ws.qslot, st));
  EGFEM_HIP_CHECK(launch_csr_matvec_perm(T, T->ws.qslot, w, out, st));
  return EGFEM_OK;
}

int egfem_matvec(egfem_tensor_t T, int which, const double* jval, int transpose, const double* x,
                 double* y, void* stream) {
  if (!T || !x || !y) return fail(EGFEM_ERR_ARG, "null argument");
  if (x == y) return fail(EGFEM_ERR_ARG, "x and y must not alias");
  const double* vals = which == 0 ? jval : (which == 1 ? T->kval : (which == 2 ? T->mval : nullptr));
  if (!vals) return fail(EGFEM_ERR_ARG, "bad matrix selector or null jval");
  hipStream_t st = (hipStream_t)stream;
  if (transpose && which == 0)
    EGFEM_HIP_CHECK(launch_csr_matvec_perm(T, vals, x, y, st));
  else
    EGFEM_HIP_CHECK(launch_csr_matvec(T, vals, x, y, st));
  return EGFEM_OK;
}

int egfem_problem_residual(egfem_tensor_t T, const egfem_problem* p, const double* u, double* F,
                           double* norm, void* stream) {
  if (!T || !p || !u || !F) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "W_h = P0 handles take the gradient coefficient (egfem_picard_grad)");
  if (F == u) return fail(EGFEM_ERR_ARG, "F must not alias u");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  EGFEM_HIP_CHECK(launch_action_problem(T, view(p), u, nullptr, 0.0, nullptr, F, T->ws.partial, st));
  if (norm) return read_norm(T, st, norm);
  return EGFEM_OK;
}

int egfem_problem_jacobian(egfem_tensor_t T, const egfem_problem* p, const double* u, double* jval,
                           double* dinv, void* stream) {
  if (!T || !p || !u || !jval) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "W_h = P0 handles take the gradient coefficient (egfem_picard_grad)");
  EGFEM_HIP_CHECK(launch_jacobian(T, u, nullptr, p->a0, p->a0_const, 1, nullptr, 1,
                                  p->add_stiffness, p->dirichlet, jval, dinv, (hipStream_t)stream));
  return EGFEM_OK;
}

void egfem_newton_opts_default(egfem_newton_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_newton = 50;
  o->max_krylov = 20000;
  o->krylov_rtol = 1e-12;
  o->forcing = 0;
  o->eta_max = 0.1;
  o->max_backtracks = 10;
  o->krylov_blocks = 0;
  o->krylov_threads = 0;
  o->timing = 0;
}

static int check_opts(const egfem_newton_opts& o) {
  if (!(o.tol >= 0.0) || o.max_newton < 0 || o.max_krylov < 1 || !(o.krylov_rtol > 0.0) ||
      !(o.eta_max > 0.0 && o.eta_max < 1.0) || o.max_backtracks < 0 || o.krylov_blocks < 0 ||
      (o.krylov_threads != 0 && o.krylov_threads != 256 && o.krylov_threads != 512 &&
       o.krylov_threads != 1024) ||
      (o.forcing != 0 && o.forcing != 1))
    return fail(EGFEM_ERR_ARG, "invalid Newton options");
  return EGFEM_OK;
}

// Eisenstat-Walker forcing term, choice 2 (gamma = 0.9, exponent 2) with the
// usual safeguards: keep eta from dropping faster than the previous term
// predicts, cap at eta_max, and do not oversolve past the outer tolerance.
static double ew_forcing(int k, double nF, double nF_prev, double eta_prev, double eta_max,
                         double tol_abs) {
  double eta;
  if (k == 0) {
    eta = eta_max;
  } else {
    eta = 0.9 * (nF / nF_prev) * (nF / nF_prev);
    const double guard = 0.9 * eta_prev * eta_prev;
    if (guard > 0.1) eta = std::max(eta, guard);
    eta = std::min(eta, eta_max);
  }
  eta = std::max(eta, 0.5 * tol_abs / nF);
  return std::min(eta, eta_max);
}

int egfem_newton(egfem_tensor_t T, const egfem_problem* p, double* u, const egfem_newton_opts* o,
                 egfem_newton_stats* s, void* stream) {
  if (!T || !p || !u) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "W_h = P0 handles take the gradient coefficient (egfem_picard_grad)");
  egfem_newton_opts opts;
  egfem_newton_opts_default(&opts);
  if (o) opts = *o;
  int rc = check_opts(opts);
  if (rc != EGFEM_OK) return rc;
  rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  hipStream_t st = (hipStream_t)stream;
  const ProblemView pv = view(p);
  egfem_newton_stats stats;
  std::memset(&stats, 0, sizeof(stats));

  LaunchTimer tm;
  if ((rc = tm.init(opts.timing != 0, st, &T->ws.timer_events)) != EGFEM_OK) return rc;
#define EGFEM_TRY(x)                    \
  do {                                  \
    if ((rc = (x)) != EGFEM_OK) return rc; \
  } while (0)

  EGFEM_HIP_CHECK(launch_mask_zero(u, p->dirichlet, T->n, st));
  EGFEM_TRY(tm.start());
  EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, nullptr, 0.0, nullptr, W.F, W.partial, st));
  EGFEM_TRY(tm.stop(&stats.t_action_ms, &stats.n_action));
  double nF0 = 0.0;
  EGFEM_TRY(read_norm(T, st, &nF0));
  stats.res0 = nF0;
  stats.res = nF0;
  int status = EGFEM_NOT_CONVERGED;
  if (!std::isfinite(nF0)) status = EGFEM_NONFINITE;
  else if (nF0 == 0.0) status = EGFEM_OK;
  double nF = nF0, nF_prev = nF0, eta = opts.eta_max;
  int k = 0;
  while (status == EGFEM_NOT_CONVERGED) {
    if (nF <= opts.tol * nF0) { status = EGFEM_OK; break; }
    if (k >= opts.max_newton) break;
    // Jacobian emission DF(u) and Jacobi diagonal
    EGFEM_TRY(tm.start());
    EGFEM_HIP_CHECK(launch_jacobian(T, u, nullptr, p->a0, p->a0_const, 1, nullptr, 1,
                                    p->add_stiffness, p->dirichlet, W.jval, W.dinv, st));
    EGFEM_TRY(tm.stop(&stats.t_jacobian_ms, &stats.n_jacobian));
    const double rtol = opts.forcing ? ew_forcing(k, nF, nF_prev, eta, opts.eta_max, opts.tol * nF0)
                                     : opts.krylov_rtol;
    eta = rtol;
    KrylovResult kr;
    // the Dirichlet rows are identity rows with zero residual: large systems
    // leave them out of the resident solve
    rc = krylov_bicgstab(T, W.jval, W.dinv, W.F, -1.0, W.delta, true, rtol, opts.max_krylov,
                         opts.krylov_blocks, &kr, st, nullptr, tm.on, opts.krylov_threads, true, p->dirichlet);
    if (rc != EGFEM_OK) return rc;
    // the full step's trial residual is enqueued behind the solve, so one
    // synchronisation reads the solve's outcome and the trial norm
    double alpha = 1.0, nFt = 0.0;
    EGFEM_TRY(tm.start());
    EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, W.delta, alpha, W.utry, W.F, W.partial, st));
    EGFEM_TRY(tm.stop(&stats.t_action_ms, &stats.n_action));
    EGFEM_TRY(read_norm(T, st, &nFt));
    if ((rc = krylov_collect(T, st, &kr)) != EGFEM_OK) return rc;
    if (tm.on) {
      stats.t_krylov_ms += kr.kernel_ms;
      ++stats.n_krylov;
    }
    stats.krylov_iters += kr.iters;
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
    if (k < EGFEM_HIST) {
      stats.krylov_hist[k] = kr.iters;
      stats.krylov_status_hist[k] = kr.status;
      stats.krylov_relres_hist[k] = kr.relres;
    }
    if (kr.status == EGFEM_NONFINITE) { status = EGFEM_NONFINITE; break; }
    // damped update u + alpha delta, residual fused with the trial iterate
    bool accepted = false;
    for (int bt = 0; bt <= opts.max_backtracks; ++bt) {
      if (bt > 0) {
        EGFEM_TRY(tm.start());
        EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, W.delta, alpha, W.utry, W.F, W.partial, st));
        EGFEM_TRY(tm.stop(&stats.t_action_ms, &stats.n_action));
        EGFEM_TRY(read_norm(T, st, &nFt));
      }
      if (std::isfinite(nFt) && nFt <= (1.0 - 1e-4 * alpha) * nF) { accepted = true; break; }
      alpha *= 0.5;
      ++stats.backtracks;
    }
    if (!accepted) {
      status = EGFEM_STAGNATED;
      // restore F at the last accepted iterate
      EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, nullptr, 0.0, nullptr, W.F, W.partial, st));
      break;
    }
    EGFEM_HIP_CHECK(launch_copy(u, W.utry, T->n, st));
    nF_prev = nF;
    nF = nFt;
    if (k < EGFEM_HIST) stats.res_hist[k] = nF;
    ++k;
  }
#undef EGFEM_TRY
  if (status == EGFEM_NOT_CONVERGED && nF <= opts.tol * nF0) status = EGFEM_OK;
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  stats.status = status;
  stats.newton_iters = k;
  stats.res = nF;
  if ((rc = tm.finish()) != EGFEM_OK) return rc;
  if (s) *s = stats;
  return status;
}

int egfem_solve(egfem_tensor_t T, const double* jval, int transpose, const double* rhs, double* x,
                double rtol, int max_iter, int* iters, double* relres, void* stream) {
  if (!T || !jval || !rhs || !x) return fail(EGFEM_ERR_ARG, "null argument");
  if (!(rtol > 0.0) || max_iter < 1) return fail(EGFEM_ERR_ARG, "rtol > 0 and max_iter >= 1 required");
  if (x == rhs) return fail(EGFEM_ERR_ARG, "x must not alias rhs");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)((T->n + 255) / 256)), dim3(256), 0, st, T->n, T->diag,
                     jval, T->ws.dinv);
  EGFEM_HIP_CHECK(hipGetLastError());
  KrylovResult kr;
  rc = krylov_bicgstab(T, jval, T->ws.dinv, rhs, 1.0, x, false, rtol, max_iter, 0, &kr, st,
                       transpose ? T->tperm : nullptr);
  if (rc != EGFEM_OK) return rc;
  if (iters) *iters = kr.iters;
  if (relres) *relres = kr.relres;
  return kr.status;
}

int egfem_solve_cg(egfem_tensor_t T, const double* jval, const double* rhs, double* x, double rtol,
                   int max_iter, int* iters, double* relres, void* stream) {
  if (!T || !jval || !rhs || !x) return fail(EGFEM_ERR_ARG, "null argument");
  if (!(rtol > 0.0) || max_iter < 1) return fail(EGFEM_ERR_ARG, "rtol > 0 and max_iter >= 1 required");
  if (x == rhs) return fail(EGFEM_ERR_ARG, "x must not alias rhs");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)((T->n + 255) / 256)), dim3(256), 0, st, T->n, T->diag,
                     jval, T->ws.dinv);
  EGFEM_HIP_CHECK(hipGetLastError());
  KrylovResult kr;
  rc = krylov_solve(KrylovMethod::kCG, T, jval, T->ws.dinv, rhs, 1.0, x, false, rtol, false, max_iter, 0, &kr,
                    st, nullptr);
  if (rc != EGFEM_OK) return rc;
  if (iters) *iters = kr.iters;
  if (relres) *relres = kr.relres;
  return kr.status;
}

void egfem_picard_opts_default(egfem_picard_opts* o) {
  if (!o) return;
  o->tol = 1e-12;
  o->max_picard = 200;
  o->max_krylov = 20000;
  o->krylov_rtol = 0.1;
  o->krylov_blocks = 0;
  o->krylov_threads = 0;
  o->timing = 0;
}

int egfem_picard(egfem_tensor_t T, const egfem_problem* p, double* u, const egfem_picard_opts* o,
                 egfem_picard_stats* s, void* stream) {
  if (!T || !p || !u) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "W_h = P0 handles take the gradient coefficient (egfem_picard_grad)");
  egfem_picard_opts opts;
  egfem_picard_opts_default(&opts);
  if (o) opts = *o;
  if (!(opts.tol >= 0.0) || opts.max_picard < 0 || opts.max_krylov < 1 || !(opts.krylov_rtol > 0.0) ||
      opts.krylov_blocks < 0 ||
      (opts.krylov_threads != 0 && opts.krylov_threads != 256 && opts.krylov_threads != 512 &&
       opts.krylov_threads != 1024))
    return fail(EGFEM_ERR_ARG, "invalid Picard options");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  hipStream_t st = (hipStream_t)stream;
  const ProblemView pv = view(p);
  egfem_picard_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  LaunchTimer tm;
  if ((rc = tm.init(opts.timing != 0, st, &T->ws.timer_events)) != EGFEM_OK) return rc;
  int n_dummy = 0;
#define EGFEM_TRY(x)                    \
  do {                                  \
    if ((rc = (x)) != EGFEM_OK) return rc; \
  } while (0)
  // u_D = 0; right-hand side d with zero Dirichlet rows
  EGFEM_HIP_CHECK(launch_mask_zero(u, p->dirichlet, T->n, st));
  if (p->load) EGFEM_HIP_CHECK(launch_copy(W.rhs, p->load, T->n, st));
  else EGFEM_HIP_CHECK(launch_fill(W.rhs, 0.0, T->n, st));
  EGFEM_HIP_CHECK(launch_mask_zero(W.rhs, p->dirichlet, T->n, st));
  EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, nullptr, 0.0, nullptr, W.F, W.partial, st));
  EGFEM_TRY(read_norm(T, st, &stats.res0));
  int status = std::isfinite(stats.res0) ? EGFEM_NOT_CONVERGED : EGFEM_NONFINITE;
  std::vector<double> part(512);
  int k = 0;
  while (status == EGFEM_NOT_CONVERGED && k < opts.max_picard) {
    // A(u^n) = [K] + T . a(u^n) with Dirichlet identity rows, and 1/diag
    EGFEM_TRY(tm.start());
    EGFEM_HIP_CHECK(launch_jacobian(T, u, nullptr, p->a0, p->a0_const, 1, nullptr, 0, p->add_stiffness,
                                    p->dirichlet, W.jval, W.dinv, st));
    EGFEM_TRY(tm.stop(&stats.t_matrix_ms, &n_dummy));
    // u^{n+1}: CG warm started from u^n
    EGFEM_HIP_CHECK(launch_copy(W.delta, u, T->n, st));
    KrylovResult kr;
    rc = krylov_solve(KrylovMethod::kCG, T, W.jval, W.dinv, W.rhs, 1.0, W.delta, false, opts.krylov_rtol,
                      true, opts.max_krylov, opts.krylov_blocks, &kr, st, nullptr, tm.on, opts.krylov_threads,
                      true);
    if (rc != EGFEM_OK) return rc;
    // relative update enqueued behind the solve: one synchronisation reads
    // the solve's outcome and the update norms; u <- u^{n+1} only after both
    // are known to be valid (an error or a non-finite step leaves u at u^n)
    hipError_t e = hipSuccess;
    const int g = launch_diff_norms(T->n, W.delta, u, W.red, st, &e);
    EGFEM_HIP_CHECK(e);
    EGFEM_HIP_CHECK(hipMemcpyAsync(part.data(), W.red, 2 * g * sizeof(double), hipMemcpyDeviceToHost, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    if ((rc = krylov_collect(T, st, &kr)) != EGFEM_OK) return rc;
    if (tm.on) stats.t_krylov_ms += kr.kernel_ms;
    stats.krylov_iters += kr.iters;
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
    if (k < EGFEM_HIST) stats.krylov_hist[k] = kr.iters;
    double dd = 0.0, xx = 0.0;
    for (int q = 0; q < g; ++q) {
      dd += part[2 * q];
      xx += part[2 * q + 1];
    }
    const double upd = xx > 0.0 ? std::sqrt(dd / xx) : 0.0;
    stats.update = upd;
    if (k < EGFEM_HIST) stats.update_hist[k] = upd;
    ++k;
    if (kr.status == EGFEM_NONFINITE || !std::isfinite(upd)) { status = EGFEM_NONFINITE; break; }
    EGFEM_HIP_CHECK(launch_copy(u, W.delta, T->n, st));
    if (upd <= opts.tol) status = EGFEM_OK;
  }
#undef EGFEM_TRY
  EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, nullptr, 0.0, nullptr, W.F, W.partial, st));
  if ((rc = read_norm(T, st, &stats.res)) != EGFEM_OK) return rc;
  stats.status = status;
  stats.picard_iters = k;
  if ((rc = tm.finish()) != EGFEM_OK) return rc;
  if (s) *s = stats;
  return status;
}

void egfem_burgers_opts_default(egfem_burgers_opts* o) {
  if (!o) return;
  o->dt = 1e-2;
  o->nu = 1.0;
  o->steps = 100;
  o->group = 0;
  o->krylov_rtol = 1e-12;
  o->max_krylov = 20000;
  o->guess = 2;
  o->krylov_blocks = 0;
  o->krylov_threads = 0;
  o->timing = 0;
}

int egfem_burgers(egfem_tensor_t T, const uint8_t* dirichlet, const double* source, int64_t source_stride,
                  double* u, const egfem_burgers_opts* o, egfem_burgers_stats* s, void* stream) {
  if (!T || !u) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->form != EGFEM_FORM_CONV) return fail(EGFEM_ERR_ARG, "Burgers steps need an EGFEM_FORM_CONV tensor");
  // W_h = P2 or I_k: the group formulation with f = (Pi_u u)^2 at the dofs of
  // W_h (the P2 dofs, or the points of the rule)
  const bool egfem_w = (T->w2 == 1 || T->w2 == 2);
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "no Burgers steps with W_h = P0");
  if (egfem_w && !(o && o->group == 1))
    return fail(EGFEM_ERR_ARG, "a W_h = P2 or I_k convection tensor takes the group formulation (group = 1)");
  egfem_burgers_opts opts;
  egfem_burgers_opts_default(&opts);
  if (o) opts = *o;
  if (!(opts.dt > 0.0) || !std::isfinite(opts.dt) || !(opts.nu >= 0.0) || !std::isfinite(opts.nu) ||
      opts.steps < 0 || opts.max_krylov < 1 || !(opts.krylov_rtol > 0.0) || opts.krylov_blocks < 0 ||
      (opts.group != 0 && opts.group != 1) || opts.guess < 0 || opts.guess > 2 ||
      (opts.krylov_threads != 0 && opts.krylov_threads != 256 && opts.krylov_threads != 512 &&
       opts.krylov_threads != 1024))
    return fail(EGFEM_ERR_ARG, "invalid Burgers options");
  if (source && source_stride < 0) return fail(EGFEM_ERR_ARG, "source_stride must be >= 0");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  // (Pi_u u)^2 is staged in the scratch vector sized for the dofs of W_h
  if (egfem_w && T->n_w > W.qslot_len) return fail(EGFEM_ERR_SHAPE, "dofs of W_h exceed the staging scratch");
  hipStream_t st = (hipStream_t)stream;
  egfem_burgers_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  LaunchTimer tm;
  if ((rc = tm.init(opts.timing != 0, st, &T->ws.timer_events)) != EGFEM_OK) return rc;
  int n_dummy = 0;
  // offline part of the run: M + dt nu K (Dirichlet identity rows, zero
  // columns) and its inverse diagonal; N^f = N contracted with 1 in j
  EGFEM_HIP_CHECK(launch_mk_combine(T, 1.0, opts.dt * opts.nu, dirichlet, W.jval, W.dinv, st));
  if (egfem_w) {
    EGFEM_HIP_CHECK(launch_fill(W.z, 1.0, T->n, st));      // u_j = 1 in the raw action gives N^f
  } else if (opts.group) {
    EGFEM_HIP_CHECK(launch_fill(W.utry, 1.0, T->n, st));
    EGFEM_HIP_CHECK(launch_slot_mode2(T, W.utry, W.qslot, st));
  }
  EGFEM_HIP_CHECK(launch_mask_zero(u, dirichlet, T->n, st));
  int status = EGFEM_OK;
  int n = 0;
  for (; n < opts.steps; ++n) {
    const double* src = source ? source + (int64_t)n * source_stride : nullptr;
    if ((rc = tm.start()) != EGFEM_OK) return rc;
    if (egfem_w) {
      // N^f (Pi_u u)^2: f on the dofs of W_h in W.qslot, raw action with u = 1
      if (T->w2 == 1) {
        EGFEM_HIP_CHECK(launch_p2_square(T, u, W.qslot, st));
      } else {
        EGFEM_HIP_CHECK(launch_iq_square(T, u, W.qslot, st));
      }
      EGFEM_HIP_CHECK(launch_action_raw(T, W.z, W.qslot, W.F, st));
    } else if (!opts.group) {
      EGFEM_HIP_CHECK(launch_action_raw(T, u, u, W.F, st));
    }
    const bool slot_group = opts.group && !egfem_w;
    EGFEM_HIP_CHECK(launch_burgers_rhs(T, slot_group, u, src, opts.dt, slot_group ? W.qslot : W.F, dirichlet,
                                       W.rhs, st));
    if ((rc = tm.stop(&stats.t_rhs_ms, &n_dummy)) != EGFEM_OK) return rc;
    // initial iterate: extrapolation over the iterates kept so far (W.delta
    // holds u^{n-1}, W.utry u^{n-2})
    EGFEM_HIP_CHECK(launch_extrapolate(T->n, std::min(opts.guess, n), u, W.delta, W.utry, st));
    KrylovResult kr;
    rc = krylov_solve(KrylovMethod::kCG, T, W.jval, W.dinv, W.rhs, 1.0, u, false, opts.krylov_rtol, false,
                      opts.max_krylov, opts.krylov_blocks, &kr, st, nullptr, tm.on, opts.krylov_threads);
    if (rc != EGFEM_OK) return rc;
    if (tm.on) stats.t_krylov_ms += kr.kernel_ms;
    stats.krylov_iters += kr.iters;
    stats.max_step_krylov = std::max(stats.max_step_krylov, kr.iters);
    if (std::isfinite(kr.relres)) stats.max_relres = std::max(stats.max_relres, kr.relres);
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
    if (n < EGFEM_HIST) stats.krylov_hist[n] = kr.iters;
    status = std::max(status, kr.status);
    if (kr.status == EGFEM_NONFINITE) {
      ++n;
      break;
    }
  }
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  stats.status = status;
  stats.steps = n;
  if ((rc = tm.finish()) != EGFEM_OK) return rc;
  if (s) *s = stats;
  return status;
}

int egfem_picard_grad(egfem_tensor_t T, const egfem_problem* p, const egfem_grad_coef* g, double* u,
                      const egfem_picard_opts* o, egfem_picard_stats* s, void* stream) {
  if (!T || !p || !g || !u) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 != 3) return fail(EGFEM_ERR_ARG, "the gradient coefficient needs a W_h = P0 handle");
  if (p->a0 || p->add_stiffness) return fail(EGFEM_ERR_ARG, "the gradient problem takes no a0 and no K term");
  if (!std::isfinite(g->c0) || !std::isfinite(g->c1) || !std::isfinite(g->q) || g->c0 < 0.0 || g->c1 < 0.0)
    return fail(EGFEM_ERR_ARG, "coefficient parameters must be finite, c0 >= 0, c1 >= 0");
  egfem_picard_opts opts;
  egfem_picard_opts_default(&opts);
  if (o) opts = *o;
  if (!(opts.tol >= 0.0) || opts.max_picard < 0 || opts.max_krylov < 1 || !(opts.krylov_rtol > 0.0) ||
      opts.krylov_blocks < 0 ||
      (opts.krylov_threads != 0 && opts.krylov_threads != 256 && opts.krylov_threads != 512 &&
       opts.krylov_threads != 1024))
    return fail(EGFEM_ERR_ARG, "invalid Picard options");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  hipStream_t st = (hipStream_t)stream;
  egfem_picard_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  LaunchTimer tm;
  if ((rc = tm.init(opts.timing != 0, st, &T->ws.timer_events)) != EGFEM_OK) return rc;
  int n_dummy = 0;
  double* a = T->e_acoef;
  std::vector<double> part(512);
  // ||F(u)|| over the free rows, F = T:(u (x) a(grad u)) - d
  auto residual_norm = [&](double* out) -> int {
    EGFEM_HIP_CHECK(launch_grad_coef(T, u, g->c0, g->c1, g->q, 0, a, nullptr, st));
    EGFEM_HIP_CHECK(launch_action_raw(T, u, a, W.F, st));
    EGFEM_HIP_CHECK(launch_mask_zero(W.F, p->dirichlet, T->n, st));
    hipError_t e = hipSuccess;
    const int ng = launch_diff_norms(T->n, W.F, W.rhs, W.red, st, &e);
    EGFEM_HIP_CHECK(e);
    EGFEM_HIP_CHECK(hipMemcpyAsync(part.data(), W.red, 2 * ng * sizeof(double), hipMemcpyDeviceToHost, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    double dd = 0.0;
    for (int q = 0; q < ng; ++q) dd += part[2 * q];
    *out = std::sqrt(dd);
    return EGFEM_OK;
  };
  // u_D = 0; right-hand side d with zero Dirichlet rows
  EGFEM_HIP_CHECK(launch_mask_zero(u, p->dirichlet, T->n, st));
  if (p->load) EGFEM_HIP_CHECK(launch_copy(W.rhs, p->load, T->n, st));
  else EGFEM_HIP_CHECK(launch_fill(W.rhs, 0.0, T->n, st));
  EGFEM_HIP_CHECK(launch_mask_zero(W.rhs, p->dirichlet, T->n, st));
  int status = EGFEM_NOT_CONVERGED;
  int k = 0;
  while (status == EGFEM_NOT_CONVERGED && k < opts.max_picard) {
    // a^n = a(Pi_grad u^n) per cell (a = 1 on the first step with start_linear)
    EGFEM_TRY_RC(tm.start());
    EGFEM_HIP_CHECK(
        launch_grad_coef(T, u, g->c0, g->c1, g->q, (k == 0 && g->start_linear) ? 1 : 0, a, nullptr, st));
    // (T . a^n) with Dirichlet identity rows and zero columns, and 1/diag
    EGFEM_HIP_CHECK(launch_jacobian(T, u, a, nullptr, 0.0, 0, nullptr, 0, 0, p->dirichlet, W.jval, W.dinv, st));
    EGFEM_TRY_RC(tm.stop(&stats.t_matrix_ms, &n_dummy));
    EGFEM_HIP_CHECK(launch_copy(W.delta, u, T->n, st));
    KrylovResult kr;
    rc = krylov_solve(KrylovMethod::kCG, T, W.jval, W.dinv, W.rhs, 1.0, W.delta, false, opts.krylov_rtol, true,
                      opts.max_krylov, opts.krylov_blocks, &kr, st, nullptr, tm.on, opts.krylov_threads, true);
    if (rc != EGFEM_OK) return rc;
    hipError_t e = hipSuccess;
    const int ng = launch_diff_norms(T->n, W.delta, u, W.red, st, &e);
    EGFEM_HIP_CHECK(e);
    EGFEM_HIP_CHECK(hipMemcpyAsync(part.data(), W.red, 2 * ng * sizeof(double), hipMemcpyDeviceToHost, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    if ((rc = krylov_collect(T, st, &kr)) != EGFEM_OK) return rc;
    if (tm.on) stats.t_krylov_ms += kr.kernel_ms;
    stats.krylov_iters += kr.iters;
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
    if (k < EGFEM_HIST) stats.krylov_hist[k] = kr.iters;
    double dd = 0.0, xx = 0.0;
    for (int q = 0; q < ng; ++q) {
      dd += part[2 * q];
      xx += part[2 * q + 1];
    }
    const double upd = xx > 0.0 ? std::sqrt(dd / xx) : 0.0;
    stats.update = upd;
    if (k < EGFEM_HIST) stats.update_hist[k] = upd;
    ++k;
    if (kr.status == EGFEM_NONFINITE || !std::isfinite(upd)) {   // u stays at the last finite iterate
      status = EGFEM_NONFINITE;
      break;
    }
    EGFEM_HIP_CHECK(launch_copy(u, W.delta, T->n, st));
    if (upd <= opts.tol) status = EGFEM_OK;
  }
  if ((rc = residual_norm(&stats.res)) != EGFEM_OK) return rc;
  stats.res0 = 0.0;
  stats.status = status;
  stats.picard_iters = k;
  if ((rc = tm.finish()) != EGFEM_OK) return rc;
  if (s) *s = stats;
  return status;
}

int egfem_newton_grad(egfem_tensor_t T, const egfem_problem* p, const egfem_grad_coef* g, double* u,
                      const egfem_newton_opts* o, egfem_newton_stats* s, void* stream) {
  if (!T || !p || !g || !u) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 != 3) return fail(EGFEM_ERR_ARG, "the gradient coefficient needs a W_h = P0 handle");
  if (p->a0 || p->add_stiffness) return fail(EGFEM_ERR_ARG, "the gradient problem takes no a0 and no K term");
  if (!std::isfinite(g->c0) || !std::isfinite(g->c1) || !std::isfinite(g->q) || g->c0 < 0.0 || g->c1 < 0.0)
    return fail(EGFEM_ERR_ARG, "coefficient parameters must be finite, c0 >= 0, c1 >= 0");
  egfem_newton_opts opts;
  egfem_newton_opts_default(&opts);
  if (o) opts = *o;
  int rc = check_opts(opts);
  if (rc != EGFEM_OK) return rc;
  rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  hipStream_t st = (hipStream_t)stream;
  egfem_newton_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  LaunchTimer tm;
  if ((rc = tm.init(opts.timing != 0, st, &T->ws.timer_events)) != EGFEM_OK) return rc;
  double* a = T->e_acoef;
  double* wv = T->e_wv;
  std::vector<double> part(256);
  // F(x) = mask(T:(x (x) a(grad x)) - d) into W.F, ||F|| to the host
  auto residual = [&](const double* x, double* nrm) -> int {
    EGFEM_TRY_RC(tm.start());
    EGFEM_HIP_CHECK(launch_grad_coef(T, x, g->c0, g->c1, g->q, 0, a, nullptr, st));
    EGFEM_HIP_CHECK(launch_action_raw(T, x, a, W.F, st));
    hipError_t e = hipSuccess;
    const int ng = launch_sub_mask_norm(T->n, W.F, W.rhs, p->dirichlet, W.red, st, &e);
    EGFEM_HIP_CHECK(e);
    EGFEM_HIP_CHECK(hipMemcpyAsync(part.data(), W.red, ng * sizeof(double), hipMemcpyDeviceToHost, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    EGFEM_TRY_RC(tm.stop(&stats.t_action_ms, &stats.n_action));
    double ss = 0.0;
    for (int q = 0; q < ng; ++q) ss += part[q];
    *nrm = std::sqrt(ss);
    return EGFEM_OK;
  };
  // CG on the symmetric Jacobian, BiCGStab if CG meets a non-positive curvature
  auto solve = [&](const double* rhs, double scale, double* x, bool x_zero, double rtol, KrylovResult* kr) -> int {
    int r2 = krylov_solve(KrylovMethod::kCG, T, W.jval, W.dinv, rhs, scale, x, x_zero, rtol, false,
                          opts.max_krylov, opts.krylov_blocks, kr, st, nullptr, tm.on, opts.krylov_threads);
    if (r2 != EGFEM_OK || kr->status != EGFEM_BREAKDOWN) return r2;
    return krylov_bicgstab(T, W.jval, W.dinv, rhs, scale, x, x_zero, rtol, opts.max_krylov, opts.krylov_blocks,
                           kr, st, nullptr, tm.on, opts.krylov_threads);
  };
  EGFEM_HIP_CHECK(launch_mask_zero(u, p->dirichlet, T->n, st));
  if (p->load) EGFEM_HIP_CHECK(launch_copy(W.rhs, p->load, T->n, st));
  else EGFEM_HIP_CHECK(launch_fill(W.rhs, 0.0, T->n, st));
  EGFEM_HIP_CHECK(launch_mask_zero(W.rhs, p->dirichlet, T->n, st));
  if (g->start_linear) {
    // u0: the Laplace solution (a = 1), solved to 1e-12 relative to d
    EGFEM_HIP_CHECK(launch_grad_coef(T, u, g->c0, g->c1, g->q, 1, a, nullptr, st));
    EGFEM_HIP_CHECK(launch_jacobian(T, u, a, nullptr, 0.0, 0, nullptr, 0, 0, p->dirichlet, W.jval, W.dinv, st));
    KrylovResult kr;
    if ((rc = solve(W.rhs, 1.0, u, true, 1e-12, &kr)) != EGFEM_OK) return rc;
    stats.krylov_iters += kr.iters;
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
  }
  double nF0 = 0.0;
  if ((rc = residual(u, &nF0)) != EGFEM_OK) return rc;
  stats.res0 = nF0;
  int status = EGFEM_NOT_CONVERGED;
  if (!std::isfinite(nF0)) status = EGFEM_NONFINITE;
  else if (nF0 == 0.0) status = EGFEM_OK;
  double nF = nF0, nF_prev = nF0, eta = opts.eta_max;
  int k = 0;
  while (status == EGFEM_NOT_CONVERGED) {
    if (nF <= opts.tol * nF0) { status = EGFEM_OK; break; }
    if (k >= opts.max_newton) break;
    // DF(u) = T . a(u) + the derivative of a(u) applied to (K^e u)_i, and 1/diag
    EGFEM_TRY_RC(tm.start());
    EGFEM_HIP_CHECK(launch_grad_coef(T, u, g->c0, g->c1, g->q, 0, a, wv, st));
    EGFEM_HIP_CHECK(launch_jacobian_grad(T, a, u, wv, p->dirichlet, W.jval, W.dinv, st));
    EGFEM_TRY_RC(tm.stop(&stats.t_jacobian_ms, &stats.n_jacobian));
    const double rtol = opts.forcing ? ew_forcing(k, nF, nF_prev, eta, opts.eta_max, opts.tol * nF0)
                                     : opts.krylov_rtol;
    eta = rtol;
    KrylovResult kr;
    if ((rc = solve(W.F, -1.0, W.delta, true, rtol, &kr)) != EGFEM_OK) return rc;
    if (tm.on) {
      stats.t_krylov_ms += kr.kernel_ms;
      ++stats.n_krylov;
    }
    stats.krylov_iters += kr.iters;
    stats.krylov_kernels |= (kr.resident ? 1 : 2) | (kr.block_precond ? 4 : 0) | (kr.overlapped ? 8 : 0);
    if (k < EGFEM_HIST) {
      stats.krylov_hist[k] = kr.iters;
      stats.krylov_status_hist[k] = kr.status;
      stats.krylov_relres_hist[k] = kr.relres;
    }
    if (kr.status == EGFEM_NONFINITE) { status = EGFEM_NONFINITE; break; }
    double alpha = 1.0, nFt = 0.0;
    bool accepted = false;
    for (int bt = 0; bt <= opts.max_backtracks; ++bt) {
      EGFEM_HIP_CHECK(launch_axpy(W.utry, u, alpha, W.delta, T->n, st));
      if ((rc = residual(W.utry, &nFt)) != EGFEM_OK) return rc;
      if (std::isfinite(nFt) && nFt <= (1.0 - 1e-4 * alpha) * nF) { accepted = true; break; }
      alpha *= 0.5;
      ++stats.backtracks;
    }
    if (!accepted) {
      status = EGFEM_STAGNATED;
      if ((rc = residual(u, &nFt)) != EGFEM_OK) return rc;   // F at the last accepted iterate
      break;
    }
    EGFEM_HIP_CHECK(launch_copy(u, W.utry, T->n, st));
    nF_prev = nF;
    nF = nFt;
    if (k < EGFEM_HIST) stats.res_hist[k] = nF;
    ++k;
  }
  if (status == EGFEM_NOT_CONVERGED && nF <= opts.tol * nF0) status = EGFEM_OK;
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  stats.status = status;
  stats.newton_iters = k;
  stats.res = nF;
  if ((rc = tm.finish()) != EGFEM_OK) return rc;
  if (s) *s = stats;
  return status;
}

int egfem_adjoint(egfem_tensor_t T, const egfem_problem* p, const double* u, const double* ubar,
                  const egfem_newton_opts* o, double* lambda, double* grad_a0, int* krylov_iters,
                  double* relres, void* stream) {
  if (!T || !p || !u || !ubar || !lambda) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2) return fail(EGFEM_ERR_ARG, "the adjoint is not available for handles with W_h != P1");
  if (lambda == u || lambda == ubar || (grad_a0 && (grad_a0 == u || grad_a0 == lambda)))
    return fail(EGFEM_ERR_ARG, "outputs must not alias inputs");
  egfem_newton_opts opts;
  egfem_newton_opts_default(&opts);
  if (o) opts = *o;
  int rc = check_opts(opts);
  if (rc != EGFEM_OK) return rc;
  rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  hipStream_t st = (hipStream_t)stream;
  // DF(u*) and its diagonal (the same for DF^T)
  EGFEM_HIP_CHECK(launch_jacobian(T, u, nullptr, p->a0, p->a0_const, 1, nullptr, 1, p->add_stiffness,
                                  p->dirichlet, W.jval, W.dinv, st));
  // right-hand side: ubar on the free nodes
  EGFEM_HIP_CHECK(launch_copy(W.rhs, ubar, T->n, st));
  EGFEM_HIP_CHECK(launch_mask_zero(W.rhs, p->dirichlet, T->n, st));
  KrylovResult kr;
  // DF's Dirichlet rows are identity rows and its Dirichlet columns zero, so
  // DF^T has the same block form and the right-hand side is zero there:
  // large systems leave those rows out of the resident solve (lambda = 0 there)
  rc = krylov_bicgstab(T, W.jval, W.dinv, W.rhs, 1.0, lambda, true, opts.krylov_rtol, opts.max_krylov,
                       opts.krylov_blocks, &kr, st, T->tperm, false, opts.krylov_threads, false, p->dirichlet);
  if (rc != EGFEM_OK) return rc;
  if (grad_a0) {
    // -sum_ij lambda_i T_ijk u_j : slot-wise (T ._2 u), then the transposed gather
    EGFEM_HIP_CHECK(launch_slot_mode2(T, u, W.qslot, st));
    EGFEM_HIP_CHECK(launch_csr_matvec_perm(T, W.qslot, lambda, grad_a0, st));
    EGFEM_HIP_CHECK(launch_scale(grad_a0, -1.0, T->n, st));
  }
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  if (krylov_iters) *krylov_iters = kr.iters;
  if (relres) *relres = kr.relres;
  return kr.status;
}

}  // extern "C"
