// Launch-shape accessors and the autotuner: candidates are timed with HIP
// events on the handle's own tensor and the fastest is kept in the handle.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "egfem_internal.h"

using namespace egfem;

namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
  }
};

// Mean duration (us) of `reps` back-to-back raw tensor actions.
int time_action(egfem_tensor_s* T, hipStream_t st, int reps, double* us) {
  Workspace& W = T->ws;
  Events ev;
  EGFEM_HIP_CHECK(hipEventCreate(&ev.a));
  EGFEM_HIP_CHECK(hipEventCreate(&ev.b));
  for (int r = 0; r < 2; ++r) EGFEM_HIP_CHECK(launch_action_raw(T, W.utry, W.delta, W.rhs, st));
  EGFEM_HIP_CHECK(hipEventRecord(ev.a, st));
  for (int r = 0; r < reps; ++r) EGFEM_HIP_CHECK(launch_action_raw(T, W.utry, W.delta, W.rhs, st));
  EGFEM_HIP_CHECK(hipEventRecord(ev.b, st));
  EGFEM_HIP_CHECK(hipEventSynchronize(ev.b));
  float ms = 0.0f;
  EGFEM_HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b));
  *us = 1000.0 * ms / reps;
  return EGFEM_OK;
}

}  // namespace

extern "C" {

int egfem_get_shape(egfem_tensor_t T, egfem_launch_shape* s) {
  if (!T || !s) return fail(EGFEM_ERR_ARG, "null argument");
  s->action_runs = T->action_runs_target;
  s->action_pipe = T->action_pipe;
  s->krylov_blocks = T->tuned_krylov_blocks;
  s->krylov_threads = T->tuned_krylov_threads;
  s->krylov_kernel = T->krylov_kernel;
  s->action_half = T->action_half;
  s->krylov_precond = T->krylov_precond;
  return EGFEM_OK;
}

int egfem_set_shape(egfem_tensor_t T, const egfem_launch_shape* s) {
  if (!T || !s) return fail(EGFEM_ERR_ARG, "null argument");
  if (s->action_runs < 0 || (s->action_pipe != 0 && s->action_pipe != 1) || s->krylov_blocks < 0 ||
      s->krylov_blocks > kMaxKrylovBlocks ||
      (s->krylov_threads != 0 && s->krylov_threads != 256 && s->krylov_threads != 512 &&
       s->krylov_threads != 1024) ||
      (s->krylov_kernel < 0 || s->krylov_kernel > 2) || (s->action_half != 0 && s->action_half != 1) ||
      s->krylov_precond < 0 || s->krylov_precond == 1 || s->krylov_precond > 32)
    return fail(EGFEM_ERR_ARG, "invalid launch shape");
  if (s->action_half && !T->vH) return fail(EGFEM_ERR_ARG, "this tensor has no symmetric half stream");
  T->action_runs_target = s->action_runs;
  T->action_pipe = s->action_pipe;
  T->tuned_krylov_blocks = s->krylov_blocks;
  T->tuned_krylov_threads = s->krylov_threads;
  T->krylov_kernel = s->krylov_kernel;
  T->action_half = s->action_half;
  T->krylov_precond = s->krylov_precond;
  return EGFEM_OK;
}

int egfem_autotune(egfem_tensor_t T, const egfem_problem* p, int what, egfem_launch_shape* best,
                   double* best_us, void* stream) {
  if (!T) return fail(EGFEM_ERR_ARG, "null handle");
  if ((what & 2) && !p) return fail(EGFEM_ERR_ARG, "Krylov tuning needs a problem");
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  Workspace& W = T->ws;
  double us_action = 0.0, us_krylov = 0.0;
  // handles with W_h != P1 run one row block per workgroup: no action shape to tune
  if ((what & 1) && !T->w2) {
    EGFEM_HIP_CHECK(launch_fill(W.utry, 0.5, T->n, st));
    EGFEM_HIP_CHECK(launch_fill(W.delta, 1.25, T->n, st));
    std::vector<int> runs = {0};
    for (int r : {8192, 4096, 2048, 1024, 512})
      if (r < T->row_blocks) runs.push_back(r);
    const int keep_runs = T->action_runs_target, keep_pipe = T->action_pipe, keep_half = T->action_half;
    T->action_half = 0;
    double best_t = DBL_MAX;
    int br = keep_runs, bp = keep_pipe;
    for (int pipe = 0; pipe <= 1; ++pipe)
      for (int r : runs) {
        if (pipe && r == 0) continue;   // pipelining needs runs of several blocks
        T->action_runs_target = r;
        T->action_pipe = pipe;
        double us = 0.0;
        if ((rc = time_action(T, st, 20, &us)) != EGFEM_OK) {
          T->action_runs_target = keep_runs;
          T->action_pipe = keep_pipe;
          T->action_half = keep_half;
          return rc;
        }
        if (us < best_t) {
          best_t = us;
          br = r;
          bp = pipe;
        }
      }
    T->action_runs_target = br;
    T->action_pipe = bp;
    T->action_half = 0;
    if (T->vH) {
      // the symmetric half stream (one row block per workgroup) against the best full-stream shape
      T->action_half = 1;
      double us = 0.0;
      if ((rc = time_action(T, st, 20, &us)) != EGFEM_OK) return rc;
      if (us < best_t) best_t = us;
      else T->action_half = 0;
    }
    us_action = best_t;
  }
  if (what & 2) {
    // DF at u = 0 of the problem, right-hand side 1 on the free rows: the time
    // per decade of residual reduction of a BiCGStab solve to 1e-8 (the block
    // preconditioner trades cost per iteration against iterations)
    EGFEM_HIP_CHECK(launch_fill(W.utry, 0.0, T->n, st));
    EGFEM_HIP_CHECK(launch_jacobian(T, W.utry, nullptr, p->a0, p->a0_const, 1, nullptr, 1, p->add_stiffness,
                                    p->dirichlet, W.jval, W.dinv, st));
    EGFEM_HIP_CHECK(launch_fill(W.rhs, 1.0, T->n, st));
    EGFEM_HIP_CHECK(launch_mask_zero(W.rhs, p->dirichlet, T->n, st));
    double best_t = DBL_MAX, best_iter_us = 0.0;
    int bb = 0, bt = 0, bk = 0;
    const int keep_kernel = T->krylov_kernel;
    for (int kernel : {0, 1})
      for (int threads : {256, 512, 1024})
        // fixed grids and the smallest grid that keeps one row per thread
        // (the largest parts of the block-Jacobi preconditioner)
        for (int blocks : {32, 64, 128, 256, 512, 1024,
                           (int)std::min<int64_t>((T->n + threads - 1) / threads, kMaxKrylovBlocks)}) {
          T->krylov_kernel = kernel;
          KrylovResult kr;
          rc = krylov_bicgstab(T, W.jval, W.dinv, W.rhs, 1.0, W.delta, true, 1e-8, 3000, blocks, &kr, st,
                               nullptr, true, threads);
          if (rc != EGFEM_OK) {
            T->krylov_kernel = keep_kernel;
            return rc;
          }
          // the register-resident kernel only where it applies (else it repeats kernel 1)
          if (kr.iters <= 0 || (kernel == 0 && !kr.resident)) continue;
          if (!(kr.relres > 0.0 && kr.relres < 1.0)) continue;
          const double per_decade = kr.kernel_ms / -std::log10(kr.relres);
          if (per_decade < best_t) {
            best_t = per_decade;
            best_iter_us = 1000.0 * kr.kernel_ms / kr.iters;
            bb = kr.blocks;
            bt = kr.threads;
            bk = kernel;
          }
        }
    T->tuned_krylov_blocks = bb;
    T->tuned_krylov_threads = bt;
    T->krylov_kernel = bk;
    us_krylov = best_iter_us;
  }
  if (best) egfem_get_shape(T, best);
  if (best_us) {
    best_us[0] = us_action;
    best_us[1] = us_krylov;
  }
  return EGFEM_OK;
}

}  // extern "C"
