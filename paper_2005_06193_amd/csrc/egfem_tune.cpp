// Launch-shape accessors and the autotuner: candidates are timed with HIP
// events on the handle's own tensor and the fastest is kept in the handle.
#include <algorithm>
#include <cfloat>
#include <chrono>
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
  s->krylov_cheb_ratio = T->krylov_cheb_ratio;
  return EGFEM_OK;
}

int egfem_set_shape(egfem_tensor_t T, const egfem_launch_shape* s) {
  if (!T || !s) return fail(EGFEM_ERR_ARG, "null argument");
  if (s->action_runs < 0 || (s->action_pipe != 0 && s->action_pipe != 1) || s->krylov_blocks < 0 ||
      s->krylov_blocks > kMaxKrylovBlocks ||
      (s->krylov_threads != 0 && s->krylov_threads != 256 && s->krylov_threads != 512 &&
       s->krylov_threads != 1024) ||
      (s->krylov_kernel < 0 || s->krylov_kernel > 2) || (s->action_half != 0 && s->action_half != 1) ||
      s->krylov_precond < 0 || s->krylov_precond == 1 || s->krylov_precond > 32 ||
      !(s->krylov_cheb_ratio == 0.0 || (s->krylov_cheb_ratio >= 2.0 && s->krylov_cheb_ratio <= 1000.0)))
    return fail(EGFEM_ERR_ARG, "invalid launch shape");
  if (s->action_half && !T->vH) return fail(EGFEM_ERR_ARG, "this tensor has no symmetric half stream");
  T->action_runs_target = s->action_runs;
  T->action_pipe = s->action_pipe;
  T->tuned_krylov_blocks = s->krylov_blocks;
  T->tuned_krylov_threads = s->krylov_threads;
  T->krylov_kernel = s->krylov_kernel;
  T->action_half = s->action_half;
  T->krylov_precond = s->krylov_precond;
  T->krylov_cheb_ratio = s->krylov_cheb_ratio > 0.0 ? s->krylov_cheb_ratio : 30.0;
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
    // The online workload itself: a damped Newton solve of problem p from
    // u = 0 to 1e-10 with Eisenstat-Walker forcing, timed per candidate grid
    // (kernel x workgroup size x workgroups; the second of two solves).
    double* u = nullptr;
    if (hipMalloc((void**)&u, std::max<int64_t>(T->n, 1) * sizeof(double)) != hipSuccess)
      return fail(EGFEM_ERR_OOM, "hipMalloc of the autotuner's iterate failed");
    egfem_newton_opts o;
    egfem_newton_opts_default(&o);
    o.tol = 1e-10;
    o.forcing = 1;
    const int keep_kernel = T->krylov_kernel, keep_blocks = T->tuned_krylov_blocks,
              keep_threads = T->tuned_krylov_threads;
    double best_t = DBL_MAX, best_iter_us = 0.0;
    int bb = keep_blocks, bt = keep_threads, bk = keep_kernel;
    for (int kernel : {0, 1})
      for (int threads : {256, 512, 1024})
        // fixed grids and the smallest grid that keeps one row per thread
        // (the largest parts of the block-Jacobi preconditioner)
        for (int blocks : {32, 64, 128, 256, 512, 1024,
                           (int)std::min<int64_t>((T->n + threads - 1) / threads, kMaxKrylovBlocks)}) {
          T->krylov_kernel = kernel;
          T->tuned_krylov_blocks = blocks;
          T->tuned_krylov_threads = threads;
          double t_solve = 0.0;
          egfem_newton_stats stt;
          bool usable = true;
          for (int rep = 0; rep < 2 && usable; ++rep) {
            if (launch_fill(u, 0.0, T->n, st) != hipSuccess) {
              rc = fail(EGFEM_ERR_HIP, "fill of the autotuner's iterate failed");
              break;
            }
            const auto t0 = std::chrono::steady_clock::now();
            const int src = egfem_newton(T, p, u, &o, &stt, stream);
            const auto t1 = std::chrono::steady_clock::now();
            if (src < 0) {
              rc = src;
              break;
            }
            t_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
            // a converged solve only; the register-resident kernel only where it ran
            // (elsewhere it repeats kernel 1)
            usable = src == EGFEM_OK && !(kernel == 0 && !(stt.krylov_kernels & 1));
          }
          if (rc != EGFEM_OK) break;
          if (!usable || stt.krylov_iters <= 0) continue;
          if (t_solve < best_t) {
            best_t = t_solve;
            best_iter_us = 0.0;
            bb = blocks;
            bt = threads;
            bk = kernel;
            best_iter_us = 1000.0 * t_solve / stt.krylov_iters;
          }
        }
    if (rc != EGFEM_OK) {
      hipFree(u);
      T->krylov_kernel = keep_kernel;
      T->tuned_krylov_blocks = keep_blocks;
      T->tuned_krylov_threads = keep_threads;
      return rc;
    }
    T->tuned_krylov_blocks = bb;
    T->tuned_krylov_threads = bt;
    T->krylov_kernel = bk;
    // the block preconditioner on that grid: Chebyshev steps x interval ratio,
    // timed the same way (the handle's own setting is among the candidates)
    const int keep_precond = T->krylov_precond;
    const double keep_ratio = T->krylov_cheb_ratio;
    int bpc = keep_precond;
    double brat = keep_ratio;
    if (keep_precond > 0) {
      for (int steps : {6, 8, 10})
        for (double ratio : {20.0, 30.0, 50.0}) {
          if (steps == keep_precond && ratio == keep_ratio) continue;   // timed above
          T->krylov_precond = steps;
          T->krylov_cheb_ratio = ratio;
          double t_solve = 0.0;
          egfem_newton_stats stt;
          bool usable = true;
          for (int rep = 0; rep < 2 && usable; ++rep) {
            if (launch_fill(u, 0.0, T->n, st) != hipSuccess) {
              rc = fail(EGFEM_ERR_HIP, "fill of the autotuner's iterate failed");
              break;
            }
            const auto t0 = std::chrono::steady_clock::now();
            const int src = egfem_newton(T, p, u, &o, &stt, stream);
            const auto t1 = std::chrono::steady_clock::now();
            if (src < 0) {
              rc = src;
              break;
            }
            t_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
            usable = src == EGFEM_OK && (stt.krylov_kernels & 4);   // the block preconditioner ran
          }
          if (rc != EGFEM_OK) break;
          if (!usable || stt.krylov_iters <= 0) continue;
          if (t_solve < best_t) {
            best_t = t_solve;
            bpc = steps;
            brat = ratio;
            best_iter_us = 1000.0 * t_solve / stt.krylov_iters;
          }
        }
    }
    hipFree(u);
    T->krylov_precond = bpc;
    T->krylov_cheb_ratio = brat;
    if (rc != EGFEM_OK) {
      T->krylov_precond = keep_precond;
      T->krylov_cheb_ratio = keep_ratio;
      return rc;
    }
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
