// Jacobi-preconditioned BiCGStab as ONE persistent cooperative launch.
//
// The linear solve of each Newton step (Sec. 4; the paper used a direct
// solve, this path uses the preconditioned BiCGStab of van der Vorst with the
// Jacobi preconditioner D = diag(J), because J = [K] + T.a + (T._2 u) diag(2u)
// is non-symmetric).  Every workgroup owns a contiguous, slot-balanced range of
// rows; all vector work is row-local.  Cross-workgroup traffic is limited to
// the vectors that matrix-vector products gather (written and read with
// agent-coherent loads/stores, so the read-only matrix stays cached in L2) and
// FP64 partial sums.  Three grid barriers per iteration, each completing one
// reduction: workgroups publish partial sums, and after the barrier every
// workgroup adds all partials in the same fixed order, so all take identical
// decisions and the result is bitwise reproducible for a fixed grid.
//
// The second product t = J D^-1 s is formed as z - alpha y with z = J D^-1 r
// (fused with v = J D^-1 p in one pass over J) and y = J D^-1 v, which removes
// the barrier that would publish D^-1 s:
//   A: v = J phat, z = J rhat_r      -> (rhat, v)                    barrier 1
//   B: alpha = rho/(rhat,v); y = J vhat; s = r - alpha v; t = z - alpha y
//                                    -> (t,s) (t,t) (rhat,s) (rhat,t) (s,s)  barrier 2
//   C: omega = (t,s)/(t,t); x += alpha phat + omega D^-1 s; r = s - omega t;
//      rho' = (rhat,s) - omega (rhat,t); beta = rho'/rho * alpha/omega;
//      p = r + beta (p - omega v); phat = D^-1 p; rhat_r = D^-1 r -> (r,r)   barrier 3
#include "egfem_internal.h"

namespace egfem {
namespace {

constexpr int kWave = 64;
constexpr unsigned kSpinCap = 1u << 24;   // bounded waits: a barrier that never completes aborts
constexpr int kGroups = 8;                // barrier arrival groups (one per XCD when dispatch is round-robin)
// ctrl layout (unsigned words, one 128-byte line each): generation, global
// arrivals, abort flag, then one arrival counter per group.
constexpr int kCtrlGen = 0, kCtrlAll = 32, kCtrlAbort = 64, kCtrlGroup = 96;
constexpr int kCtrlWords = kCtrlGroup + 32 * kGroups;
static_assert(kCtrlWords <= kCtrlWordsMax, "barrier control block too small");

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
  double *r, *rhat, *p, *v, *s, *t, *z;     // row-local
  double *phat, *rh, *vh;                   // gathered by other workgroups (agent-coherent)
  const int32_t* krow;
  double* red;              // [kRedSlots][8][G]
  unsigned* ctrl;           // kCtrlWords
  double rtol;
  int max_iter;
  double* out;              // [0] status [1] iterations [2] relres [3] ||b||
};

// Agent-coherent accessors for data exchanged between workgroups.
__device__ __forceinline__ double ld_sh(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier with epoch counting (no counter resets).  Every wave first
// waits until its own stores are complete (s_waitcnt vmcnt(0)); data shared
// across workgroups is written and read with agent-coherent accesses, so no
// cache write-back or invalidation is needed.  Arrivals are counted per group
// of workgroups, the last of each group arrives at the global counter, the
// last global arrival publishes the new epoch, everyone else polls it.
// Returns true when the grid aborted (a wait exceeded kSpinCap).
__device__ bool grid_barrier(unsigned* ctrl, unsigned epoch, int* sh_abort) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x;
    const unsigned ng = G < (unsigned)kGroups ? G : (unsigned)kGroups;
    const unsigned grp = blockIdx.x % ng;
    const unsigned gsz = (G - grp + ng - 1) / ng;   // workgroups b < G with b % ng == grp
    int ab = (int)__hip_atomic_load(ctrl + kCtrlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!ab) {
      const unsigned prev = __hip_atomic_fetch_add(ctrl + kCtrlGroup + 32 * grp, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      bool last = false;
      if (prev == (epoch + 1) * gsz - 1) {
        const unsigned prev2 = __hip_atomic_fetch_add(ctrl + kCtrlAll, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        last = (prev2 == (epoch + 1) * ng - 1);
      }
      if (last) {
        __hip_atomic_store(ctrl + kCtrlGen, epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        unsigned spins = 0;
        while (__hip_atomic_load(ctrl + kCtrlGen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= epoch) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins >= kSpinCap) {
            __hip_atomic_store(ctrl + kCtrlAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ab = 1;
            break;
          }
          if ((spins & 1023u) == 0 &&
              __hip_atomic_load(ctrl + kCtrlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ab = 1;
            break;
          }
        }
      }
    }
    *sh_abort = ab;
  }
  __syncthreads();
  return *sh_abort != 0;
}

constexpr int kMaxRed = 8;   // values per reduction

// Deterministic block sum of up to kMaxRed values; results broadcast to all threads.
template <int NT>
__device__ void block_sum(double (&v)[kMaxRed], int m, double* sh) {
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
    sh[kMaxRed * NW + threadIdx.x] = acc;
  }
  __syncthreads();
  for (int q = 0; q < m; ++q) v[q] = sh[kMaxRed * NW + q];
  __syncthreads();
}

// Publish this workgroup's block sums into reduction slot `slot`, pass the
// grid barrier, then add the G partials of every value in a fixed order.
template <int NT>
__device__ bool grid_reduce(const KArgs& A, int slot, double (&v)[kMaxRed], int m, double* sh,
                            int* sh_abort, unsigned& epoch) {
  const unsigned G = gridDim.x;
  block_sum<NT>(v, m, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < m; ++q) st_sh(A.red + ((size_t)slot * kMaxRed + q) * G + blockIdx.x, v[q]);
  if (grid_barrier(A.ctrl, epoch++, sh_abort)) return true;
  double w[kMaxRed];
  for (int q = 0; q < m; ++q) {
    const double* src = A.red + ((size_t)slot * kMaxRed + q) * G;
    double acc = 0.0;
    for (unsigned g = threadIdx.x; g < G; g += NT) acc += ld_sh(src + g);
    w[q] = acc;
  }
  block_sum<NT>(w, m, sh);
  for (int q = 0; q < m; ++q) v[q] = w[q];
  return false;
}

// Rows [rb, re) of this workgroup, L lanes per row: calls f(i, (J x1)_i, (J x2)_i)
// on lane 0 of each row's group (x2 may be null).  x1 / x2 are gathered with
// agent-coherent loads when SH.
template <int NT, int L, bool SH, typename Fn>
__device__ __forceinline__ void spmv_rows(const KArgs& A, int rb, int re, const double* __restrict__ x1,
                                          const double* __restrict__ x2, Fn f) {
  constexpr int RPP = NT / L;   // rows per pass
  const int sub = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  for (int base = rb; base < re; base += RPP) {
    const int i = base + sub;
    double acc1 = 0.0, acc2 = 0.0;
    if (i < re) {
      const int e = A.rowptr[i + 1];
      for (int s = A.rowptr[i] + lane; s < e; s += L) {
        const double a = A.perm ? A.val[A.perm[s]] : A.val[s];
        const int c = A.col[s];
        acc1 = fma(a, SH ? ld_sh(x1 + c) : x1[c], acc1);
        if (x2) acc2 = fma(a, SH ? ld_sh(x2 + c) : x2[c], acc2);
      }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
      acc1 += __shfl_xor(acc1, off, L);
      acc2 += __shfl_xor(acc2, off, L);
    }
    if (i < re && lane == 0) f(i, acc1, acc2);
  }
}

template <int NT, int L>
__global__ __launch_bounds__(NT) void k_bicgstab(KArgs A) {
  __shared__ double sh[kMaxRed * (NT / kWave) + kMaxRed];
  __shared__ int sh_abort;
  const int rb = A.krow[blockIdx.x], re = A.krow[blockIdx.x + 1];
  const int tid = threadIdx.x;
  double red[kMaxRed];
  bool abort = false;
  int status = EGFEM_NOT_CONVERGED;
  int it = 0;
  unsigned epoch = 0;
  double rnorm = 0.0, bnorm = 0.0;
#define ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0

  // ---- setup: r = b - J x, rhat = p = r, phat = rh = D^-1 r ---------------
  ZERO_RED();
  if (A.x_zero) {
    for (int i = rb + tid; i < re; i += NT) {
      const double bi = A.rhs_scale * A.rhs[i];
      const double di = A.dinv[i] * bi;
      A.x[i] = 0.0;
      A.r[i] = bi;
      A.rhat[i] = bi;
      A.p[i] = bi;
      st_sh(A.phat + i, di);
      st_sh(A.rh + i, di);
      red[0] = fma(bi, bi, red[0]);
      red[1] = fma(bi, bi, red[1]);
    }
  } else {
    spmv_rows<NT, L, false>(A, rb, re, A.x, nullptr, [&](int i, double Jx, double) {
      const double bi = A.rhs_scale * A.rhs[i];
      const double ri = bi - Jx;
      const double di = A.dinv[i] * ri;
      A.r[i] = ri;
      A.rhat[i] = ri;
      A.p[i] = ri;
      st_sh(A.phat + i, di);
      st_sh(A.rh + i, di);
      red[0] = fma(ri, ri, red[0]);
      red[1] = fma(bi, bi, red[1]);
    });
  }
  abort = grid_reduce<NT>(A, 0, red, 2, sh, &sh_abort, epoch);
  double rho = red[0];
  rnorm = sqrt(red[0]);
  bnorm = sqrt(red[1]);
  const double r0norm = rnorm;
  int restarts = 0;
  int slot = 1;

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
        // lost bi-orthogonality: restart once from the current residual
        // (rhat = r, p = r, phat = D^-1 r = rh, rho = (r, r))
        if (restarts++ >= 1) { status = EGFEM_BREAKDOWN; break; }
        ZERO_RED();
        for (int i = rb + tid; i < re; i += NT) {
          const double ri = A.r[i];
          A.rhat[i] = ri;
          A.p[i] = ri;
          st_sh(A.phat + i, ld_sh(A.rh + i));
          red[0] = fma(ri, ri, red[0]);
        }
        if ((abort = grid_reduce<NT>(A, 7, red, 1, sh, &sh_abort, epoch))) break;
        rho = red[0];
        continue;
      }
      // ---- A: v = J phat, z = J rh ; (rhat, v) ----------------------------
      ZERO_RED();
      spmv_rows<NT, L, true>(A, rb, re, A.phat, A.rh, [&](int i, double vi, double zi) {
        A.v[i] = vi;
        A.z[i] = zi;
        st_sh(A.vh + i, A.dinv[i] * vi);
        red[0] = fma(A.rhat[i], vi, red[0]);
      });
      if ((abort = grid_reduce<NT>(A, slot, red, 1, sh, &sh_abort, epoch))) break;
      slot = slot % 6 + 1;
      const double rv = red[0];
      if (rv == 0.0 || !isfinite(rv)) { status = isfinite(rv) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
      const double alpha = rho / rv;
      // ---- B: y = J vh ; s = r - alpha v ; t = z - alpha y ------------------
      ZERO_RED();
      spmv_rows<NT, L, true>(A, rb, re, A.vh, nullptr, [&](int i, double yi, double) {
        const double si = fma(-alpha, A.v[i], A.r[i]);
        const double ti = fma(-alpha, yi, A.z[i]);
        const double hi = A.rhat[i];
        A.s[i] = si;
        A.t[i] = ti;
        red[0] = fma(ti, si, red[0]);
        red[1] = fma(ti, ti, red[1]);
        red[2] = fma(hi, si, red[2]);
        red[3] = fma(hi, ti, red[3]);
        red[4] = fma(si, si, red[4]);
      });
      if ((abort = grid_reduce<NT>(A, slot, red, 5, sh, &sh_abort, epoch))) break;
      slot = slot % 6 + 1;
      ++it;
      if (sqrt(red[4]) <= A.rtol * bnorm) {
        for (int i = rb + tid; i < re; i += NT) A.x[i] = fma(alpha, ld_sh(A.phat + i), A.x[i]);
        rnorm = sqrt(red[4]);
        status = EGFEM_OK;
        break;
      }
      if (red[1] == 0.0 || !isfinite(red[1])) { status = isfinite(red[1]) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
      const double omega = red[0] / red[1];
      if (omega == 0.0) { status = EGFEM_BREAKDOWN; break; }
      const double rho_new = fma(-omega, red[3], red[2]);
      const double beta = (rho_new / rho) * (alpha / omega);
      rho = rho_new;
      // ---- C: x, r, p, phat, rh ; (r, r) -----------------------------------
      ZERO_RED();
      for (int i = rb + tid; i < re; i += NT) {
        const double di = A.dinv[i];
        const double si = A.s[i];
        const double xi = fma(alpha, ld_sh(A.phat + i), fma(omega, di * si, A.x[i]));
        const double ri = fma(-omega, A.t[i], si);
        const double pi = fma(beta, fma(-omega, A.v[i], A.p[i]), ri);
        A.x[i] = xi;
        A.r[i] = ri;
        A.p[i] = pi;
        st_sh(A.phat + i, di * pi);
        st_sh(A.rh + i, di * ri);
        red[0] = fma(ri, ri, red[0]);
      }
      if ((abort = grid_reduce<NT>(A, slot, red, 1, sh, &sh_abort, epoch))) break;
      slot = slot % 6 + 1;
      rnorm = sqrt(red[0]);
    }
  }
#undef ZERO_RED
  if (blockIdx.x == 0 && tid == 0) {
    A.out[0] = abort ? (double)EGFEM_ERR_HIP : (double)status;
    A.out[1] = (double)it;
    A.out[2] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    A.out[3] = bnorm;
  }
}

template <int NT, int L>
hipError_t launch_NL(const KArgs& A, unsigned G, hipStream_t st) {
  void* args[] = {(void*)&A};
  return hipLaunchCooperativeKernel((const void*)k_bicgstab<NT, L>, dim3(G), dim3(NT), args, 0, st);
}

template <int NT, int L>
int max_coresident_NL() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bicgstab<NT, L>, NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

// Dispatch over the compiled (threads, lanes-per-row) shapes.
template <int NT>
struct ShapeNT {
  static hipError_t launch(int L, const KArgs& A, unsigned G, hipStream_t st) {
    switch (L) {
      case 4: return launch_NL<NT, 4>(A, G, st);
      case 8: return launch_NL<NT, 8>(A, G, st);
      case 16: return launch_NL<NT, 16>(A, G, st);
      case 32: return launch_NL<NT, 32>(A, G, st);
      default: return launch_NL<NT, 64>(A, G, st);
    }
  }
  static int cap(int L) {
    switch (L) {
      case 4: return max_coresident_NL<NT, 4>();
      case 8: return max_coresident_NL<NT, 8>();
      case 16: return max_coresident_NL<NT, 16>();
      case 32: return max_coresident_NL<NT, 32>();
      default: return max_coresident_NL<NT, 64>();
    }
  }
};

hipError_t launch_shape(int NT, int L, const KArgs& A, unsigned G, hipStream_t st) {
  if (NT == 256) return ShapeNT<256>::launch(L, A, G, st);
  if (NT == 512) return ShapeNT<512>::launch(L, A, G, st);
  return ShapeNT<1024>::launch(L, A, G, st);
}

int cap_shape(int NT, int L) {
  if (NT == 256) return ShapeNT<256>::cap(L);
  if (NT == 512) return ShapeNT<512>::cap(L);
  return ShapeNT<1024>::cap(L);
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
                    KrylovResult* res, hipStream_t st, const int32_t* perm, bool timed, int threads) {
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  const int NT = (threads == 256 || threads == 512 || threads == 1024) ? threads : kKrylovThreads;
  const int cap = cap_shape(NT, T->krylov_lanes);
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
  EGFEM_HIP_CHECK(launch_fill_u32(W.ctrl, 0u, kCtrlWords, st));
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
  A.z = W.z;
  A.phat = W.phat;
  A.rh = W.rh;
  A.vh = W.vh;
  A.krow = W.krow;
  A.red = W.red;
  A.ctrl = W.ctrl;
  A.rtol = rtol;
  A.max_iter = max_iter;
  A.out = W.kout;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (timed) {
    EGFEM_HIP_CHECK(hipEventCreate(&ev0));
    EGFEM_HIP_CHECK(hipEventCreate(&ev1));
    EGFEM_HIP_CHECK(hipEventRecord(ev0, st));
  }
  const hipError_t e = launch_shape(NT, T->krylov_lanes, A, (unsigned)G, st);
  if (e != hipSuccess) {
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    return fail(EGFEM_ERR_HIP, std::string("cooperative launch failed: ") + hipGetErrorString(e));
  }
  if (timed) EGFEM_HIP_CHECK(hipEventRecord(ev1, st));
  EGFEM_HIP_CHECK(hipMemcpyAsync(W.host_kout, W.kout, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  if (timed) {
    float ms = 0.0f;
    EGFEM_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
    res->kernel_ms = ms;
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
  }
  const double* o = W.host_kout;
  res->status = (int)o[0];
  res->iters = (int)o[1];
  res->relres = o[2];
  res->bnorm = o[3];
  res->blocks = G;
  res->threads = NT;
  if (res->status == EGFEM_ERR_HIP) return fail(EGFEM_ERR_HIP, "Krylov grid barrier timed out");
  return EGFEM_OK;
}

}  // namespace egfem
