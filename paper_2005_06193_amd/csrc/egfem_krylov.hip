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
#include "egfem_device.h"

namespace egfem {
namespace {

using dev::KArgs;

struct LaunchArgs {
  KArgs A;
  const int32_t* krow;      // row partition [G+1]
  unsigned* ctrl;
  double* red;
  double* out;              // [0] status [1] iterations [2] relres [3] ||b||
};

// One team spanning the whole grid.
template <int NT, int RS>
__global__ __launch_bounds__(NT) void k_bicgstab(LaunchArgs P) {
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_abort;
  dev::Team tm{blockIdx.x, gridDim.x, P.ctrl, P.red, 0u};
  const int rb = P.krow[blockIdx.x], re = P.krow[blockIdx.x + 1];
  const dev::KOut o = dev::team_bicgstab<NT, row_L(RS), row_K(RS)>(tm, P.A, rb, re, sh, &sh_abort);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.out[0] = o.abort ? (double)EGFEM_ERR_HIP : (double)o.status;
    P.out[1] = (double)o.iters;
    P.out[2] = o.bnorm > 0.0 ? o.rnorm / o.bnorm : 0.0;
    P.out[3] = o.bnorm;
  }
}

// Register-resident form: one thread per row, rows of at most K entries.
constexpr int kResidentRow = 8;

template <int NT, int K>
__global__ __launch_bounds__(NT) void k_bicgstab_reg(LaunchArgs P) {
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_abort;
  dev::Team tm{blockIdx.x, gridDim.x, P.ctrl, P.red, 0u};
  const int rb = P.krow[blockIdx.x], re = P.krow[blockIdx.x + 1];
  const dev::KOut o = dev::team_bicgstab_reg<NT, K>(tm, P.A, rb, re, sh, &sh_abort);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.out[0] = o.abort ? (double)EGFEM_ERR_HIP : (double)o.status;
    P.out[1] = (double)o.iters;
    P.out[2] = o.bnorm > 0.0 ? o.rnorm / o.bnorm : 0.0;
    P.out[3] = o.bnorm;
  }
}

template <int NT, int K>
hipError_t launch_reg_NK(const LaunchArgs& A, unsigned G, hipStream_t st) {
  void* args[] = {(void*)&A};
  return hipLaunchCooperativeKernel((const void*)k_bicgstab_reg<NT, K>, dim3(G), dim3(NT), args, 0, st);
}

template <int NT, int K>
int max_coresident_reg_NK() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bicgstab_reg<NT, K>, NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

template <int NT, int RS>
hipError_t launch_NL(const LaunchArgs& A, unsigned G, hipStream_t st) {
  void* args[] = {(void*)&A};
  return hipLaunchCooperativeKernel((const void*)k_bicgstab<NT, RS>, dim3(G), dim3(NT), args, 0, st);
}

template <int NT, int RS>
int max_coresident_NL() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bicgstab<NT, RS>, NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

// Dispatch over the compiled (threads, row shape) pairs.
template <int NT>
struct ShapeNT {
  static hipError_t launch(int rs, const LaunchArgs& A, unsigned G, hipStream_t st) {
    switch (rs) {
      case 0: return launch_NL<NT, 0>(A, G, st);
      case 1: return launch_NL<NT, 1>(A, G, st);
      case 2: return launch_NL<NT, 2>(A, G, st);
      case 3: return launch_NL<NT, 3>(A, G, st);
      case 4: return launch_NL<NT, 4>(A, G, st);
      case 5: return launch_NL<NT, 5>(A, G, st);
      case 6: return launch_NL<NT, 6>(A, G, st);
      case 7: return launch_NL<NT, 7>(A, G, st);
      default: return launch_NL<NT, 8>(A, G, st);
    }
  }
  // register-resident form: rows of at most kResidentRow entries
  static hipError_t launch_reg(const LaunchArgs& A, unsigned G, hipStream_t st) {
    return launch_reg_NK<NT, kResidentRow>(A, G, st);
  }
  static int cap_reg() { return max_coresident_reg_NK<NT, kResidentRow>(); }
  static int cap(int rs) {
    switch (rs) {
      case 0: return max_coresident_NL<NT, 0>();
      case 1: return max_coresident_NL<NT, 1>();
      case 2: return max_coresident_NL<NT, 2>();
      case 3: return max_coresident_NL<NT, 3>();
      case 4: return max_coresident_NL<NT, 4>();
      case 5: return max_coresident_NL<NT, 5>();
      case 6: return max_coresident_NL<NT, 6>();
      case 7: return max_coresident_NL<NT, 7>();
      default: return max_coresident_NL<NT, 8>();
    }
  }
};

hipError_t launch_shape(int NT, int L, const LaunchArgs& A, unsigned G, hipStream_t st) {
  if (NT == 256) return ShapeNT<256>::launch(L, A, G, st);
  if (NT == 512) return ShapeNT<512>::launch(L, A, G, st);
  return ShapeNT<1024>::launch(L, A, G, st);
}

int cap_shape(int NT, int L) {
  if (NT == 256) return ShapeNT<256>::cap(L);
  if (NT == 512) return ShapeNT<512>::cap(L);
  return ShapeNT<1024>::cap(L);
}

hipError_t launch_shape_reg(int NT, const LaunchArgs& A, unsigned G, hipStream_t st) {
  if (NT == 256) return ShapeNT<256>::launch_reg(A, G, st);
  if (NT == 512) return ShapeNT<512>::launch_reg(A, G, st);
  return ShapeNT<1024>::launch_reg(A, G, st);
}

int cap_shape_reg(int NT) {
  if (NT == 256) return ShapeNT<256>::cap_reg();
  if (NT == 512) return ShapeNT<512>::cap_reg();
  return ShapeNT<1024>::cap_reg();
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
  if (threads == 0) threads = T->tuned_krylov_threads;
  if (blocks <= 0) blocks = T->tuned_krylov_blocks;
  const int NT = (threads == 256 || threads == 512 || threads == 1024) ? threads : kKrylovThreads;
  const int cap = cap_shape(NT, T->krylov_rs);
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
    int most = 0;
    for (int g = 0; g < G; ++g) most = std::max(most, kr[g + 1] - kr[g]);
    W.krow_maxrows = most;
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.krow, kr.data(), kr.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    W.krow_blocks = G;
  }
  EGFEM_HIP_CHECK(launch_fill_u32(W.ctrl, 0u, dev::kCtrlWords, st));
  LaunchArgs P;
  KArgs& A = P.A;
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
  A.rtol = rtol;
  A.max_iter = max_iter;
  P.krow = W.krow;
  P.ctrl = W.ctrl;
  P.red = W.red;
  P.out = W.kout;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (timed) {
    EGFEM_HIP_CHECK(hipEventCreate(&ev0));
    EGFEM_HIP_CHECK(hipEventCreate(&ev1));
    EGFEM_HIP_CHECK(hipEventRecord(ev0, st));
  }
  // register-resident form when every workgroup's rows fit its threads, rows
  // hold at most kResidentRow entries, and the grid is co-resident for it
  const int L = T->krylov_lanes;
  // (columns are held as 32-bit byte offsets: n < 2^28)
  const bool resident = T->krylov_kernel == 0 && T->max_row_slots <= kResidentRow &&
                        W.krow_maxrows <= NT && T->n < (int64_t(1) << 28) && G <= cap_shape_reg(NT);
  const hipError_t e = resident ? launch_shape_reg(NT, P, (unsigned)G, st)
                                : launch_shape(NT, T->krylov_rs, P, (unsigned)G, st);
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
  res->resident = resident;
  if (res->status == EGFEM_ERR_HIP) return fail(EGFEM_ERR_HIP, "Krylov grid barrier timed out");
  return EGFEM_OK;
}

}  // namespace egfem
