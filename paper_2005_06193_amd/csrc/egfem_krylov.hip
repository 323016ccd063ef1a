// Jacobi-preconditioned BiCGStab as ONE persistent cooperative launch.
//
// The linear solve of each Newton step (Sec. 4; the paper used a direct
// solve, this path uses the preconditioned BiCGStab of van der Vorst with the
// Jacobi preconditioner D = diag(J), because J = K + T.a + (T._2 u) diag(2u)
// is non-symmetric).  Every workgroup owns a contiguous, slot-balanced range of
// rows; all vector work is row-local and the only cross-workgroup traffic is
// (a) the gathered entries of the two preconditioned search vectors in the
// matrix-vector products and (b) FP64 dot products.  Each iteration has four
// grid barriers; every barrier also completes one reduction: workgroups write
// their partial sums, and after the barrier each workgroup adds all partials
// in the same fixed order, so every workgroup takes identical decisions and
// the result is bitwise reproducible for a fixed grid.
//
//   per iteration (rho = (rhat, r) carried):
//     v = J phat                     -> (rhat, v)            barrier 1
//     alpha = rho / (rhat, v); s = r - alpha v; shat = D^-1 s -> (s, s)   barrier 2
//     t = J shat                     -> (t,s) (t,t) (rhat,s) (rhat,t)    barrier 3
//     omega = (t,s)/(t,t); x += alpha phat + omega shat; r = s - omega t
//     rho' = (rhat,s) - omega (rhat,t); beta = rho'/rho * alpha/omega
//     p = r + beta (p - omega v); phat = D^-1 p -> (r, r)   barrier 4
#include "egfem_internal.h"

namespace egfem {
namespace {

constexpr int kWave = 64;
constexpr unsigned kSpinCap = 1u << 24;   // bounded waits: a barrier that never completes aborts

struct KArgs {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int32_t* perm;      // non-null: use val[perm[s]] (transposed operator)
  const double* dinv;
  const double* rhs;
  double rhs_scale;
  double* x;
  int x_zero;
  double *r, *rhat, *p, *v, *s, *t, *phat, *shat;
  const int32_t* krow;
  double* red;              // [kRedSlots][4][G]
  unsigned* ctrl;           // [0] count, [1] generation, [2] abort
  double rtol;
  int max_iter;
  double* out;              // [0] status [1] iterations [2] relres [3] ||b||
};

// Grid barrier (generation counter).  Every thread publishes its global
// writes with an agent-scope release before the workgroup barrier; thread 0
// arrives; after the generation flips, every thread acquires.  Returns true
// when the grid aborted (a wait exceeded kSpinCap).
__device__ bool grid_barrier(unsigned* ctrl, unsigned G, int* sh_abort) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* count = ctrl;
    unsigned* gen = ctrl + 1;
    unsigned* abortf = ctrl + 2;
    int ab = (int)__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!ab) {
      const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == G - 1) {
        __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        unsigned spins = 0;
        while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins >= kSpinCap) {
            __hip_atomic_store(abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ab = 1;
            break;
          }
          if ((spins & 1023u) == 0 &&
              __hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ab = 1;
            break;
          }
        }
      }
    }
    *sh_abort = ab;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *sh_abort != 0;
}

// Deterministic block sum of up to 4 values; results broadcast to all threads.
template <int NT>
__device__ void block_sum4(double (&v)[4], int m, double* sh) {
  constexpr int NW = NT / kWave;
  for (int q = 0; q < m; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[q * NW + threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)m) {
    double acc = 0.0;
    for (int w = 0; w < NW; ++w) acc += sh[threadIdx.x * NW + w];
    sh[4 * NW + threadIdx.x] = acc;
  }
  __syncthreads();
  for (int q = 0; q < m; ++q) v[q] = sh[4 * NW + q];
  __syncthreads();
}

// Publish this workgroup's block sums into reduction slot `slot`, pass the
// grid barrier, then add the G partials of every value in a fixed order.
template <int NT>
__device__ bool grid_reduce(const KArgs& A, int slot, double (&v)[4], int m, double* sh,
                            int* sh_abort) {
  const unsigned G = gridDim.x;
  block_sum4<NT>(v, m, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < m; ++q) A.red[((size_t)slot * 4 + q) * G + blockIdx.x] = v[q];
  if (grid_barrier(A.ctrl, G, sh_abort)) return true;
  double w[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < m; ++q) {
    const double* src = A.red + ((size_t)slot * 4 + q) * G;
    double acc = 0.0;
    for (unsigned g = threadIdx.x; g < G; g += NT) acc += src[g];
    w[q] = acc;
  }
  block_sum4<NT>(w, m, sh);
  for (int q = 0; q < m; ++q) v[q] = w[q];
  return false;
}

// y_i = (J x)_i for the rows [rb, re) of this workgroup, L lanes per row.
// Calls f(i, y_i) on lane 0 of each row's group.
template <int NT, int L, typename Fn>
__device__ __forceinline__ void spmv_rows(const KArgs& A, int rb, int re, const double* __restrict__ x,
                                          Fn f) {
  constexpr int RPP = NT / L;   // rows per pass
  const int sub = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  for (int base = rb; base < re; base += RPP) {
    const int i = base + sub;
    double acc = 0.0;
    if (i < re) {
      const int e = A.rowptr[i + 1];
      for (int s = A.rowptr[i] + lane; s < e; s += L) {
        const double a = A.perm ? A.val[A.perm[s]] : A.val[s];
        acc = fma(a, x[A.col[s]], acc);
      }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
    if (i < re && lane == 0) f(i, acc);
  }
}

template <int NT, int L>
__global__ __launch_bounds__(NT) void k_bicgstab(KArgs A) {
  __shared__ double sh[4 * (NT / kWave) + 8];
  __shared__ int sh_abort;
  const int rb = A.krow[blockIdx.x], re = A.krow[blockIdx.x + 1];
  const int tid = threadIdx.x;
  double red[4];
  bool abort = false;
  int status = EGFEM_NOT_CONVERGED;
  int it = 0;
  double rnorm = 0.0, bnorm = 0.0;

  // ---- setup: r = b - J x, rhat = p = r, phat = D^-1 p -------------------
  red[0] = red[1] = red[2] = red[3] = 0.0;
  if (A.x_zero) {
    for (int i = rb + tid; i < re; i += NT) {
      const double bi = A.rhs_scale * A.rhs[i];
      A.x[i] = 0.0;
      A.r[i] = bi;
      A.rhat[i] = bi;
      A.p[i] = bi;
      A.phat[i] = A.dinv[i] * bi;
      red[0] = fma(bi, bi, red[0]);
      red[1] = fma(bi, bi, red[1]);
    }
  } else {
    spmv_rows<NT, L>(A, rb, re, A.x, [&](int i, double Jx) {
      const double bi = A.rhs_scale * A.rhs[i];
      const double ri = bi - Jx;
      A.r[i] = ri;
      A.rhat[i] = ri;
      A.p[i] = ri;
      A.phat[i] = A.dinv[i] * ri;
      red[0] = fma(ri, ri, red[0]);
      red[1] = fma(bi, bi, red[1]);
    });
  }
  abort = grid_reduce<NT>(A, 0, red, 2, sh, &sh_abort);
  double rho = red[0];
  rnorm = sqrt(red[0]);
  bnorm = sqrt(red[1]);
  const double r0norm = rnorm;
  int restarts = 0;
  double alpha = 0.0, omega = 0.0;

  if (!abort && bnorm == 0.0) {
    for (int i = rb + tid; i < re; i += NT) A.x[i] = 0.0;
    status = EGFEM_OK;
    rnorm = 0.0;
  } else {
    while (!abort) {
      if (!isfinite(rnorm) || !isfinite(rho)) { status = EGFEM_NONFINITE; break; }
      if (rnorm <= A.rtol * bnorm) { status = EGFEM_OK; break; }
      if (it >= A.max_iter) { status = EGFEM_NOT_CONVERGED; break; }
      if (fabs(rho) <= 1e-15 * r0norm * rnorm) {
        // breakdown of the bi-orthogonality: restart once from the current residual
        if (restarts++ >= 1) { status = EGFEM_BREAKDOWN; break; }
        red[0] = red[1] = red[2] = red[3] = 0.0;
        for (int i = rb + tid; i < re; i += NT) {
          const double ri = A.r[i];
          A.rhat[i] = ri;
          A.p[i] = ri;
          A.phat[i] = A.dinv[i] * ri;
          red[0] = fma(ri, ri, red[0]);
        }
        if ((abort = grid_reduce<NT>(A, 5, red, 1, sh, &sh_abort))) break;
        rho = red[0];
        continue;
      }
      // v = J phat ; (rhat, v)
      red[0] = red[1] = red[2] = red[3] = 0.0;
      spmv_rows<NT, L>(A, rb, re, A.phat, [&](int i, double vi) {
        A.v[i] = vi;
        red[0] = fma(A.rhat[i], vi, red[0]);
      });
      if ((abort = grid_reduce<NT>(A, 1, red, 1, sh, &sh_abort))) break;
      const double rv = red[0];
      if (rv == 0.0 || !isfinite(rv)) { status = isfinite(rv) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
      alpha = rho / rv;
      // s = r - alpha v ; shat = D^-1 s ; (s, s)
      red[0] = 0.0;
      for (int i = rb + tid; i < re; i += NT) {
        const double si = fma(-alpha, A.v[i], A.r[i]);
        A.s[i] = si;
        A.shat[i] = A.dinv[i] * si;
        red[0] = fma(si, si, red[0]);
      }
      if ((abort = grid_reduce<NT>(A, 2, red, 1, sh, &sh_abort))) break;
      const double snorm = sqrt(red[0]);
      ++it;
      if (snorm <= A.rtol * bnorm) {
        for (int i = rb + tid; i < re; i += NT) A.x[i] = fma(alpha, A.phat[i], A.x[i]);
        rnorm = snorm;
        status = EGFEM_OK;
        break;
      }
      // t = J shat ; (t,s) (t,t) (rhat,s) (rhat,t)
      red[0] = red[1] = red[2] = red[3] = 0.0;
      spmv_rows<NT, L>(A, rb, re, A.shat, [&](int i, double ti) {
        A.t[i] = ti;
        const double si = A.s[i], hi = A.rhat[i];
        red[0] = fma(ti, si, red[0]);
        red[1] = fma(ti, ti, red[1]);
        red[2] = fma(hi, si, red[2]);
        red[3] = fma(hi, ti, red[3]);
      });
      if ((abort = grid_reduce<NT>(A, 3, red, 4, sh, &sh_abort))) break;
      if (red[1] == 0.0 || !isfinite(red[1])) { status = isfinite(red[1]) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
      omega = red[0] / red[1];
      const double rho_new = fma(-omega, red[3], red[2]);
      if (omega == 0.0) { status = EGFEM_BREAKDOWN; break; }
      const double beta = (rho_new / rho) * (alpha / omega);
      rho = rho_new;
      // x, r, p, phat ; (r, r)
      red[0] = 0.0;
      for (int i = rb + tid; i < re; i += NT) {
        const double xi = fma(alpha, A.phat[i], fma(omega, A.shat[i], A.x[i]));
        const double ri = fma(-omega, A.t[i], A.s[i]);
        const double pi = fma(beta, fma(-omega, A.v[i], A.p[i]), ri);
        A.x[i] = xi;
        A.r[i] = ri;
        A.p[i] = pi;
        A.phat[i] = A.dinv[i] * pi;
        red[0] = fma(ri, ri, red[0]);
      }
      if ((abort = grid_reduce<NT>(A, 4, red, 1, sh, &sh_abort))) break;
      rnorm = sqrt(red[0]);
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    A.out[0] = abort ? (double)EGFEM_ERR_HIP : (double)status;
    A.out[1] = (double)it;
    A.out[2] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    A.out[3] = bnorm;
  }
}

template <int L>
hipError_t launch_L(const KArgs& A, unsigned G, hipStream_t st) {
  void* args[] = {(void*)&A};
  return hipLaunchCooperativeKernel((const void*)k_bicgstab<kKrylovThreads, L>, dim3(G),
                                    dim3(kKrylovThreads), args, 0, st);
}

template <int L>
int max_coresident() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bicgstab<kKrylovThreads, L>,
                                               kKrylovThreads, 0);
  return per_cu * cus;
}

}  // namespace

// Slot-balanced partition of the rows over G workgroups.
static void make_partition(const egfem_tensor_s* T, int G, std::vector<int32_t>& kr) {
  kr.assign(G + 1, 0);
  const int64_t N = T->n;
  const int64_t S = T->slots;
  int64_t i = 0;
  for (int g = 1; g < G; ++g) {
    const int64_t target = (S * g) / G;
    while (i < N && T->h_rowptr[i] < target) ++i;
    kr[g] = (int32_t)i;
  }
  kr[G] = (int32_t)N;
}

int krylov_bicgstab(egfem_tensor_s* T, const double* jval, const double* dinv, const double* rhs,
                    double rhs_scale, double* x, bool x_zero, double rtol, int max_iter, int blocks,
                    KrylovResult* res, hipStream_t st, const int32_t* perm) {
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  int cap = 0;
  switch (T->lanes_per_row) {
    case 4: cap = max_coresident<4>(); break;
    case 8: cap = max_coresident<8>(); break;
    case 16: cap = max_coresident<16>(); break;
    case 32: cap = max_coresident<32>(); break;
    default: cap = max_coresident<64>(); break;
  }
  if (cap <= 0) return fail(EGFEM_ERR_HIP, "Krylov kernel cannot be resident");
  int G = blocks;
  if (G <= 0) {
    // about 64 rows per workgroup at least, one workgroup per CU at most by default
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    G = (int)std::min<int64_t>((T->n + 63) / 64, (int64_t)cus);
  }
  G = std::max(1, std::min({G, cap, kMaxKrylovBlocks, (int)T->n}));
  if (W.krow_blocks != G) {
    std::vector<int32_t> kr;
    make_partition(T, G, kr);
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.krow, kr.data(), kr.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    W.krow_blocks = G;
  }
  EGFEM_HIP_CHECK(launch_fill_u32(W.ctrl, 0u, 4, st));
  KArgs A;
  A.n = T->n;
  A.rowptr = T->rowptr;
  A.col = T->col;
  A.val = jval;
  A.perm = perm;
  A.dinv = dinv;
  A.rhs = rhs;
  A.rhs_scale = rhs_scale;
  A.x = x;
  A.x_zero = x_zero ? 1 : 0;
  A.r = W.r;
  A.rhat = W.rhat;
  A.p = W.p;
  A.v = W.v;
  A.s = W.s;
  A.t = W.t;
  A.phat = W.phat;
  A.shat = W.shat;
  A.krow = W.krow;
  A.red = W.red;
  A.ctrl = W.ctrl;
  A.rtol = rtol;
  A.max_iter = max_iter;
  A.out = W.kout;
  hipError_t e;
  switch (T->lanes_per_row) {
    case 4: e = launch_L<4>(A, (unsigned)G, st); break;
    case 8: e = launch_L<8>(A, (unsigned)G, st); break;
    case 16: e = launch_L<16>(A, (unsigned)G, st); break;
    case 32: e = launch_L<32>(A, (unsigned)G, st); break;
    default: e = launch_L<64>(A, (unsigned)G, st); break;
  }
  if (e != hipSuccess) return fail(EGFEM_ERR_HIP, std::string("cooperative launch failed: ") + hipGetErrorString(e));
  EGFEM_HIP_CHECK(hipMemcpyAsync(W.host_kout, W.kout, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  const double* o = W.host_kout;
  res->status = (int)o[0];
  res->iters = (int)o[1];
  res->relres = o[2];
  res->bnorm = o[3];
  res->blocks = G;
  if (res->status == EGFEM_ERR_HIP) return fail(EGFEM_ERR_HIP, "Krylov grid barrier timed out");
  return EGFEM_OK;
}

}  // namespace egfem
