// Preconditioned BiCGStab and CG, each as ONE persistent cooperative launch.
//
// The linear solve of each Newton step (Sec. 4; the paper used a direct
// solve, this path uses the preconditioned BiCGStab of van der Vorst, because
// J = [K] + T.a + (T._2 u) diag(2u) is non-symmetric; the Picard and Burgers
// matrices are SPD and take CG).  Every workgroup owns a set of rows: a
// contiguous, slot-balanced range, or, for the register-resident kernels with
// the block-Jacobi preconditioner, one part of a recursive coordinate
// bisection (a compact patch of the mesh).  All vector work is row-local.
// Cross-workgroup traffic is limited to the vectors that matrix-vector
// products gather (written and read with agent-coherent loads/stores, so the
// read-only matrix stays cached in L2) and FP64 partial sums.  Reductions
// complete at grid barriers: workgroups publish partial sums, and after the
// barrier every workgroup adds all partials in the same fixed order, so all
// take identical decisions and the result is bitwise reproducible for a
// fixed grid.
//
// With M the preconditioner (D = diag(J), or the workgroup-local block-Jacobi
// operator, which needs no communication between workgroups), the second
// product t = J M^-1 s is formed as z - alpha y with z = J M^-1 r (fused with
// v = J M^-1 p in one pass over J) and y = J M^-1 v, which removes the barrier
// that would publish M^-1 s:
//   A: v = J phat, z = J rhat_r      -> (rhat, v)                    barrier 1
//   B: alpha = rho/(rhat,v); y = J vhat; s = r - alpha v; t = z - alpha y
//                                    -> (t,s) (t,t) (rhat,s) (rhat,t) (s,s)  barrier 2
//   C: omega = (t,s)/(t,t); x += alpha phat + omega M^-1 s; r = s - omega t;
//      rho' = (rhat,s) - omega (rhat,t); beta = rho'/rho * alpha/omega;
//      p = r + beta (p - omega v); phat = M^-1 p; rhat_r = M^-1 r -> (r,r)   barrier 3
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "egfem_device.h"
#include "egfem_krylov_ov.h"

namespace egfem {
namespace {

using dev::KArgs;

struct LaunchArgs {
  KArgs A;
  dev::OvArgs ov;           // flagged exchange of the overlapped block-Jacobi BiCGStab
  const int32_t* krow;      // row partition [G+1]
  const int32_t* nbr;       // [G][kMaxNbr + 1] neighbour lists (count, ranks), or null
  unsigned* ctrl;
  double* red;
  double* out;              // [0] status [1] iterations [2] relres [3] ||b||
};

// One team spanning the whole grid; the kernel writes its outcome to P.out.
__device__ void write_out(const LaunchArgs& P, const dev::KOut& o) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.out[0] = o.abort ? (double)EGFEM_ERR_HIP : (double)o.status;
    P.out[1] = (double)o.iters;
    P.out[2] = o.bnorm > 0.0 ? o.rnorm / o.bnorm : 0.0;
    P.out[3] = o.bnorm;
  }
}

#define EGFEM_TEAM_PROLOGUE()                                   \
  __shared__ double sh[dev::kShWords<NT>];                      \
  __shared__ int sh_abort;                                      \
  dev::Team tm{blockIdx.x, gridDim.x, P.ctrl, P.red, 0u};       \
  if (P.nbr) tm.nbr = P.nbr + (size_t)blockIdx.x * (dev::kMaxNbr + 1); \
  const int rb = P.krow[blockIdx.x], re = P.krow[blockIdx.x + 1]

// Streaming BiCGStab (row shape code RS).
template <int NT, int RS>
__global__ __launch_bounds__(NT) void k_bicgstab(LaunchArgs P) {
  EGFEM_TEAM_PROLOGUE();
  write_out(P, dev::team_bicgstab<NT, row_L(RS), row_K(RS)>(tm, P.A, rb, re, sh, &sh_abort));
}

// Streaming conjugate gradients (row shape code RS).
template <int NT, int RS>
__global__ __launch_bounds__(NT) void k_pcg(LaunchArgs P) {
  EGFEM_TEAM_PROLOGUE();
  write_out(P, dev::team_pcg<NT, row_L(RS), row_K(RS)>(tm, P.A, rb, re, sh, &sh_abort));
}

// Register-resident forms: one thread per row, rows of at most K entries,
// workgroups of at most kResidentMaxThreads threads; the barrier-form BiCGStab
// also at 1024 threads (a lane then holds at most 128 VGPRs: it keeps its
// shadow residual in memory and its reduction totals in scalar registers).
constexpr int kResidentMaxThreads = 512;

// KW > 0: rows of up to K + KW entries, the KW past the first K in LDS (the
// 1024-thread form for 3D meshes, whose rows hold up to 15 entries).
// LX: products from LDS (the part's own rows and its ghosts staged per product).
template <int NT, int K, int KW = 0, bool LX = false>
__global__ __launch_bounds__(NT) void k_bicgstab_reg(LaunchArgs P) {
  EGFEM_TEAM_PROLOGUE();
  // at 1024 threads the point-to-point synchronisation's registers do not fit
  // beside the row's: the team barrier stands in for it
  if constexpr (NT > kResidentMaxThreads) tm.nbr = nullptr;
  write_out(P, dev::team_bicgstab_reg<NT, K, KW, LX>(tm, P.A, rb, re, sh, &sh_abort));
}

// Overlapped block-Jacobi BiCGStab on a compact partition (one thread per
// row, rows of at most kResidentRow entries, at most NT ghost columns per
// part); the grid's last workgroup aggregates the reductions.
template <int NT>
__global__ __launch_bounds__(NT) void k_bicgstab_ov(LaunchArgs P) {
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_state[2];
  if (threadIdx.x == 0) sh_state[1] = 0;
  dev::AggRed ar{blockIdx.x, gridDim.x - 1, P.ov.salt, P.ov.part, P.ov.tot, P.ov.exit_word,
                 P.ctrl + dev::kCtrlAbort};
  if (blockIdx.x == gridDim.x - 1) {
    dev::agg_serve<NT>(ar);
    return;
  }
  const int rb = P.krow[blockIdx.x], re = P.krow[blockIdx.x + 1];
  const dev::KOut o = dev::team_bicgstab_ov<NT, kResidentRow>(ar, P.A, P.ov, rb, re, sh, sh_state);
  if (blockIdx.x == 0 && threadIdx.x == 0)   // every reduction is complete: release the aggregator
    __hip_atomic_store(P.ov.exit_word, (uint64_t)dev::ll_flag(P.ov.salt, dev::kLLEpochMask) << 32,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  write_out(P, o);
}

// Overlapped block-Jacobi conjugate gradients (same arrangement).
template <int NT>
__global__ __launch_bounds__(NT) void k_pcg_ov(LaunchArgs P) {
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_state[2];
  if (threadIdx.x == 0) sh_state[1] = 0;
  dev::AggRed ar{blockIdx.x, gridDim.x - 1, P.ov.salt, P.ov.part, P.ov.tot, P.ov.exit_word,
                 P.ctrl + dev::kCtrlAbort};
  if (blockIdx.x == gridDim.x - 1) {
    dev::agg_serve<NT>(ar);
    return;
  }
  const int rb = P.krow[blockIdx.x], re = P.krow[blockIdx.x + 1];
  const dev::KOut o = dev::team_pcg_ov<NT, kResidentRow>(ar, P.A, P.ov, rb, re, sh, sh_state);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(P.ov.exit_word, (uint64_t)dev::ll_flag(P.ov.salt, dev::kLLEpochMask) << 32,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  write_out(P, o);
}

template <int NT, int K>
__global__ __launch_bounds__(NT) void k_pcg_reg(LaunchArgs P) {
  EGFEM_TEAM_PROLOGUE();
  write_out(P, dev::team_pcg_reg<NT, K>(tm, P.A, rb, re, sh, &sh_abort));
}
#undef EGFEM_TEAM_PROLOGUE

// Kernel for (method, resident, row shape) at workgroup size NT.
template <int NT, int RS>
const void* streaming_kernel(KrylovMethod m) {
  return m == KrylovMethod::kCG ? (const void*)k_pcg<NT, RS> : (const void*)k_bicgstab<NT, RS>;
}

// Resident kernels exist for rows of at most kResidentRow entries, and at
// 1024 threads (BiCGStab) also for wide rows of up to kResidentRow + kWideRow;
// null where there is none.
template <int NT>
const void* kernel_NT(KrylovMethod m, bool resident, int rs, bool wide, bool lx) {
  if constexpr (NT <= kResidentMaxThreads) {
    if (resident && (wide || lx)) return nullptr;
    if (resident)
      return m == KrylovMethod::kCG ? (const void*)k_pcg_reg<NT, kResidentRow>
                                    : (const void*)k_bicgstab_reg<NT, kResidentRow>;
  } else {
    // 1024 threads: the barrier-form BiCGStab only (fits the 128 registers a
    // lane has at that size, no spill), for the free-row partition
    if (resident) {
      if (m != KrylovMethod::kBiCGStab) return nullptr;
      if (lx)
        return wide ? (const void*)k_bicgstab_reg<NT, kResidentRow, kWideRow, true>
                    : (const void*)k_bicgstab_reg<NT, kResidentRow, 0, true>;
      return wide ? (const void*)k_bicgstab_reg<NT, kResidentRow, kWideRow>
                  : (const void*)k_bicgstab_reg<NT, kResidentRow>;
    }
  }
  switch (rs) {
    case 0: return streaming_kernel<NT, 0>(m);
    case 1: return streaming_kernel<NT, 1>(m);
    case 2: return streaming_kernel<NT, 2>(m);
    case 3: return streaming_kernel<NT, 3>(m);
    case 4: return streaming_kernel<NT, 4>(m);
    case 5: return streaming_kernel<NT, 5>(m);
    case 6: return streaming_kernel<NT, 6>(m);
    case 7: return streaming_kernel<NT, 7>(m);
    default: return streaming_kernel<NT, 8>(m);
  }
}

const void* kernel_for(int NT, KrylovMethod m, bool resident, int rs, bool wide = false, bool lx = false) {
  if (NT == 256) return kernel_NT<256>(m, resident, rs, wide, lx);
  if (NT == 512) return kernel_NT<512>(m, resident, rs, wide, lx);
  return kernel_NT<1024>(m, resident, rs, wide, lx);
}

// Workgroups of this kernel that can be resident at once on the current
// device (queried once per kernel, workgroup size and device).
int coresident(const void* kern, int NT) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, int>, int> cache;
  int dev = 0;
  hipGetDevice(&dev);
  const auto key = std::make_tuple(kern, NT, dev);
  {
    std::lock_guard<std::mutex> lk(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  int per_cu = 0, cus = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = per_cu * cus;
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

int krylov_solve(KrylovMethod method, egfem_tensor_s* T, const double* jval, const double* dinv,
                 const double* rhs, double rhs_scale, double* x, bool x_zero, double rtol, bool rel_r0,
                 int max_iter, int blocks, KrylovResult* res, hipStream_t st, const int32_t* perm, bool timed,
                 int threads, bool defer, const uint8_t* skip_rows) {
  int rc = ensure_workspace(T);
  if (rc != EGFEM_OK) return rc;
  Workspace& W = T->ws;
  if (threads == 0) threads = T->tuned_krylov_threads;
  if (blocks <= 0) blocks = T->tuned_krylov_blocks;
  // Free-row resident BiCGStab: rows marked in skip_rows (the Newton system's
  // Dirichlet rows: identity rows, zero right-hand side, zero columns, so
  // also for the transposed operator) are left out of the solve (their x is
  // 0), so that one row per thread of 1024-thread workgroups covers systems
  // above the 256/512-thread resident capacity.  Rows of up to
  // kResidentRow + kWideRow entries (3D meshes) run this form only.
  const bool wide = T->max_row_slots > kResidentRow;
  const bool free_ok = skip_rows && x_zero && method == KrylovMethod::kBiCGStab && T->krylov_kernel != 1 &&
                       T->max_row_slots <= kResidentRow + kWideRow && T->krylov_precond > 0 &&
                       !T->h_coords.empty() && T->n < (int64_t(1) << 28);
  int64_t n_free = T->n;
  if (free_ok) {
    // the mask as it is now (it is compared, not trusted, on every call)
    std::vector<uint8_t> hm((size_t)T->n);
    EGFEM_HIP_CHECK(hipMemcpyAsync(hm.data(), skip_rows, hm.size(), hipMemcpyDeviceToHost, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    if (W.crow_skip != hm || W.crow_skip_dev != skip_rows) {
      W.crow_skip.swap(hm);
      W.crow_skip_dev = skip_rows;
      W.crow_blocks = 0;   // a free-row partition built for another mask is stale
    }
    n_free = 0;
    for (uint8_t b : W.crow_skip) n_free += b ? 0 : 1;
  }
  if (threads == 0 && blocks <= 0 && T->krylov_kernel != 1 && T->max_row_slots <= kResidentRow + kWideRow &&
      T->n <= (int64_t)256 * kMaxKrylovBlocks) {
    // untuned, register-resident: 256-thread workgroups, one row per thread,
    // as few as that allows (largest block-Jacobi parts); kept only when the
    // grid is co-resident; above that, or for wide rows, 1024-thread
    // workgroups on the free rows
    const int g = (int)((T->n + 255) / 256);
    const int gf = (int)((n_free + 1023) / 1024);
    if (!wide && g <= coresident(kernel_for(256, method, true, 0), 256)) {
      threads = 256;
      blocks = g;
    } else if (free_ok && n_free > 0 && gf <= coresident(kernel_for(1024, method, true, 0, wide), 1024)) {
      threads = 1024;
      blocks = gf;
    }
  }
  const int NT = (threads == 256 || threads == 512 || threads == 1024) ? threads : kKrylovThreads;
  // the free-row partition serves the 1024-thread resident form only
  const bool free_rows = free_ok && NT == 1024 && n_free > 0;
  if (free_rows) blocks = std::max(blocks, (int)((n_free + NT - 1) / NT));
  const int cap = coresident(kernel_for(NT, method, false, T->krylov_rs), NT);
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
  if (free_rows) G = std::min<int64_t>(G, n_free);   // every part holds a free row
  if (W.krow_blocks != G) {
    std::vector<int32_t> kr;
    make_partition(T, G, kr);
    int most = 0;
    for (int g = 0; g < G; ++g) most = std::max(most, kr[g + 1] - kr[g]);
    W.krow_maxrows = most;
    // neighbour lists: the other workgroups owning a column of this one's rows
    std::vector<int32_t> nb((size_t)G * (kMaxNbrLists + 1), 0);
    for (int g = 0; g < G; ++g) {
      int32_t* lst = nb.data() + (size_t)g * (kMaxNbrLists + 1);
      int cnt = 0;
      for (int32_t s = T->h_rowptr[kr[g]]; s < T->h_rowptr[kr[g + 1]] && cnt >= 0; ++s) {
        const int32_t c = T->h_col[s];
        if (c >= kr[g] && c < kr[g + 1]) continue;
        const int owner = (int)(std::upper_bound(kr.begin(), kr.end(), c) - kr.begin()) - 1;
        bool seen = false;
        for (int q = 0; q < cnt; ++q) seen = seen || lst[1 + q] == owner;
        if (seen) continue;
        if (cnt == kMaxNbrLists) cnt = -1;   // too many: the team barrier
        else lst[1 + cnt++] = owner;
      }
      lst[0] = cnt;
    }
    uniform_neighbor_lists(nb, G);
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.knbr, nb.data(), nb.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.krow, kr.data(), kr.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    W.krow_blocks = G;
  }
  // register-resident form when every workgroup's rows fit its threads, rows
  // hold at most kResidentRow entries, and the grid is co-resident for it
  // (columns are held as 32-bit byte offsets: n < 2^28)
  const void* kreg = kernel_for(NT, method, true, 0, wide);   // null where there is none
  // (1024 threads: BiCGStab only, on the free rows or on every row)
  const bool resident_ok = kreg && T->krylov_kernel != 1 && T->max_row_slots <= kResidentRow + kWideRow &&
                           T->n < (int64_t(1) << 28) && G <= coresident(kreg, NT);
  // block-Jacobi preconditioner: the resident kernels on a compact partition
  // (of the free rows at 1024 threads)
  bool block = resident_ok && T->krylov_precond > 0 && !T->h_coords.empty() && (n_free + G - 1) / G <= NT;
  if (block && (W.crow_blocks != G || W.crow_free != free_rows)) {
    CompactPartition cp;
    if ((rc = make_compact_partition(T->dim, T->h_coords.data(), T->n, T->h_rowptr.data(), T->h_col.data(), G,
                                     cp, free_rows ? W.crow_skip.data() : nullptr)) != EGFEM_OK)
      return rc;
    W.crow_free = free_rows;
    if (!W.crlist) {
      if (hipMalloc((void**)&W.crow, ((size_t)kMaxKrylovBlocks + 1) * sizeof(int32_t)) != hipSuccess ||
          hipMalloc((void**)&W.cnbr, (size_t)kMaxKrylovBlocks * (kMaxNbrLists + 1) * sizeof(int32_t)) !=
              hipSuccess ||
          hipMalloc((void**)&W.crlist, std::max<size_t>(T->n, 1) * sizeof(int32_t)) != hipSuccess ||
          hipMalloc((void**)&W.ckloc, std::max<size_t>(T->slots, 1) * sizeof(int16_t)) != hipSuccess)
        return fail(EGFEM_ERR_OOM, "hipMalloc of the compact partition failed");
      T->device_bytes += (int64_t)(((size_t)kMaxKrylovBlocks + 1) * 4 +
                                   (size_t)kMaxKrylovBlocks * (kMaxNbrLists + 1) * 4 + (size_t)T->n * 4 +
                                   (size_t)T->slots * 2);
    }
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.crow, cp.kr.data(), cp.kr.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.cnbr, cp.nbr.data(), cp.nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                   st));
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.crlist, cp.rlist.data(), cp.rlist.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipMemcpyAsync(W.ckloc, cp.kloc.data(), cp.kloc.size() * sizeof(int16_t),
                                   hipMemcpyHostToDevice, st));
    EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    W.crow_blocks = G;
    W.crow_maxrows = cp.maxrows;
    // ghosts of every part (its rows' out-of-part columns, ascending) and the
    // LDS position of every entry: part-local (>= 0) or -1 - ghost index
    std::vector<int16_t> kext(cp.kloc.begin(), cp.kloc.end());
    std::vector<int32_t> gptr(1, 0), gcol;
    int maxghost = 0;
    std::vector<int32_t> gl;
    for (int g = 0; g < G; ++g) {
      gl.clear();
      for (int32_t q = cp.kr[g]; q < cp.kr[g + 1]; ++q) {
        const int32_t rr = cp.rlist[q];
        for (int32_t sl = T->h_rowptr[rr]; sl < T->h_rowptr[rr + 1]; ++sl)
          if (cp.kloc[sl] < 0) gl.push_back(T->h_col[sl]);
      }
      std::sort(gl.begin(), gl.end());
      gl.erase(std::unique(gl.begin(), gl.end()), gl.end());
      for (int32_t q = cp.kr[g]; q < cp.kr[g + 1]; ++q) {
        const int32_t rr = cp.rlist[q];
        for (int32_t sl = T->h_rowptr[rr]; sl < T->h_rowptr[rr + 1]; ++sl)
          if (cp.kloc[sl] < 0)
            kext[sl] = (int16_t)(-1 - (int)(std::lower_bound(gl.begin(), gl.end(), T->h_col[sl]) - gl.begin()));
      }
      maxghost = std::max(maxghost, (int)gl.size());
      gcol.insert(gcol.end(), gl.begin(), gl.end());
      gptr.push_back((int32_t)gcol.size());
    }
    W.crow_maxghost = maxghost;
    if (maxghost <= 1024) {   // int16 positions, at most one ghost per thread
      if (!W.ckext) {
        if (hipMalloc((void**)&W.ckext, std::max<size_t>(T->slots, 1) * sizeof(int16_t)) != hipSuccess ||
            hipMalloc((void**)&W.cgptr, ((size_t)kMaxKrylovBlocks + 1) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void**)&W.cgcol, std::max<size_t>(T->slots, 1) * sizeof(int32_t)) != hipSuccess)
          return fail(EGFEM_ERR_OOM, "hipMalloc of the ghost lists failed");
        T->device_bytes += (int64_t)T->slots * 6 + ((int64_t)kMaxKrylovBlocks + 1) * 4;
      }
      EGFEM_HIP_CHECK(hipMemcpyAsync(W.ckext, kext.data(), kext.size() * sizeof(int16_t), hipMemcpyHostToDevice, st));
      EGFEM_HIP_CHECK(hipMemcpyAsync(W.cgptr, gptr.data(), gptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      if (!gcol.empty())
        EGFEM_HIP_CHECK(hipMemcpyAsync(W.cgcol, gcol.data(), gcol.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                       st));
      EGFEM_HIP_CHECK(hipStreamSynchronize(st));
    }
  }
  block = block && W.crow_maxrows <= NT;   // one thread per row
  // the 1024-thread form takes its products from LDS where every part's
  // ghosts fit its threads
  const void* klx = (block && NT == 1024 && W.ckext && W.crow_maxghost <= NT && T->krylov_kernel != 2)
                        ? kernel_for(NT, method, true, 0, wide, true) : nullptr;
  const bool lx = klx && G <= coresident(klx, NT);
  if (lx) kreg = klx;
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
  A.rel_r0 = rel_r0 ? 1 : 0;
  P.krow = block ? W.crow : W.krow;
  P.nbr = block ? W.cnbr : W.knbr;
  if (block) {
    A.rlist = W.crlist;
    A.kloc = W.ckloc;
    A.cheb_steps = T->krylov_precond;
    A.cheb_ratio = T->krylov_cheb_ratio;
  }
  if (lx) {
    A.kext = W.ckext;
    A.gptr = W.cgptr;
    A.gcol = W.cgcol;
  }
  P.ctrl = W.ctrl;
  P.red = W.red;
  P.out = W.kout;
  if (W.kpend.active) {   // an outcome never collected (an earlier call returned early)
    if (W.kpend.ev0) hipEventDestroy(W.kpend.ev0);
    if (W.kpend.ev1) hipEventDestroy(W.kpend.ev1);
    W.kpend = KrylovPending();
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (timed) {
    EGFEM_HIP_CHECK(hipEventCreate(&ev0));
    EGFEM_HIP_CHECK(hipEventCreate(&ev1));
    EGFEM_HIP_CHECK(hipEventRecord(ev0, st));
  }
  const bool resident = block || (resident_ok && W.krow_maxrows <= NT);
  // the overlapped block-Jacobi BiCGStab (flag-in-data synchronisation) where
  // the block preconditioner runs, unless the shape asks for the barrier form
  const void* kov = nullptr;
  if (block && NT <= 512 && T->krylov_kernel == 0 && W.crow_maxghost <= NT && W.ckext) {
    if (method == KrylovMethod::kBiCGStab)
      kov = NT == 256 ? (const void*)k_bicgstab_ov<256> : (const void*)k_bicgstab_ov<512>;
    else
      kov = NT == 256 ? (const void*)k_pcg_ov<256> : (const void*)k_pcg_ov<512>;
  }
  const bool overlapped = kov && G + 1 <= coresident(kov, NT);   // plus the aggregating workgroup
  // Flagged words of the overlapped kernel: the published vectors [3][n][2]
  // and the reduction words (partials [2][4][2][kMaxKrylovBlocks], totals, exit
  // word), in one buffer that only this kernel writes.  A word is trusted when
  // its flag carries the launch's salt (1 .. 4095, advanced per launch), so
  // the buffer is zeroed when allocated and again whenever the salt wraps:
  // every flag it holds then comes from a distinct earlier launch of this
  // handle.
  const size_t ll_vec_words = (size_t)6 * std::max<int64_t>(T->n, 1);
  const size_t ll_red_words = (size_t)2 * dev::kAggValues * 2 * kMaxKrylovBlocks + 2 * dev::kAggValues * 2 + 8;
  if (overlapped && !W.llv) {
    const size_t bytes = (ll_vec_words + ll_red_words) * sizeof(uint64_t);
    if (hipMalloc((void**)&W.llv, bytes) != hipSuccess)
      return fail(EGFEM_ERR_OOM, "hipMalloc of the flagged words failed");
    T->device_bytes += (int64_t)bytes;
    W.ll_salt = 0;
  }
  if (overlapped) {
    if (W.ll_salt == 0 || W.ll_salt == 4095u)
      EGFEM_HIP_CHECK(launch_fill_u32(reinterpret_cast<unsigned*>(W.llv), 0u,
                                      (int64_t)(2 * (ll_vec_words + ll_red_words)), st));
    W.ll_salt = W.ll_salt % 4095u + 1u;
    P.ov.llv = W.llv;
    P.ov.kext = W.ckext;
    P.ov.gptr = W.cgptr;
    P.ov.gcol = W.cgcol;
    P.ov.part = W.llv + ll_vec_words;
    P.ov.tot = P.ov.part + (size_t)2 * dev::kAggValues * 2 * kMaxKrylovBlocks;
    P.ov.exit_word = P.ov.tot + 2 * dev::kAggValues * 2;
    P.ov.salt = W.ll_salt;
  }
  if (free_rows && block) {
    // rows left out are never written: x = 0 there, and the published
    // vectors hold 0 where the solve gathers them with zero matrix entries
    EGFEM_HIP_CHECK(launch_fill(x, 0.0, T->n, st));
    EGFEM_HIP_CHECK(launch_fill(W.phat, 0.0, T->n, st));
    EGFEM_HIP_CHECK(launch_fill(W.rh, 0.0, T->n, st));
    EGFEM_HIP_CHECK(launch_fill(W.vh, 0.0, T->n, st));
  }
  const void* kern = overlapped ? kov : (resident ? kreg : kernel_for(NT, method, false, T->krylov_rs));
  void* args[] = {(void*)&P};
  const hipError_t e = hipLaunchCooperativeKernel(kern, dim3((unsigned)(overlapped ? G + 1 : G)), dim3((unsigned)NT),
                                                   args, 0, st);
  if (e != hipSuccess) {
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    return fail(EGFEM_ERR_HIP, std::string("cooperative launch failed: ") + hipGetErrorString(e));
  }
  if (timed) EGFEM_HIP_CHECK(hipEventRecord(ev1, st));
  EGFEM_HIP_CHECK(hipMemcpyAsync(W.host_kout, W.kout, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  KrylovPending& q = W.kpend;
  q.active = true;
  q.ev0 = ev0;
  q.ev1 = ev1;
  q.G = G;
  q.NT = NT;
  q.resident = resident;
  q.block = block;
  q.overlapped = overlapped;
  if (defer) return EGFEM_OK;
  return krylov_collect(T, st, res);
}

int krylov_collect(egfem_tensor_s* T, hipStream_t st, KrylovResult* res) {
  Workspace& W = T->ws;
  KrylovPending& q = W.kpend;
  if (!q.active) return fail(EGFEM_ERR_ARG, "no Krylov solve in flight");
  q.active = false;
  const hipError_t e = hipStreamSynchronize(st);
  if (q.ev0) {
    float ms = 0.0f;
    if (e == hipSuccess && hipEventElapsedTime(&ms, q.ev0, q.ev1) == hipSuccess) res->kernel_ms = ms;
    hipEventDestroy(q.ev0);
    hipEventDestroy(q.ev1);
    q.ev0 = q.ev1 = nullptr;
  }
  if (e != hipSuccess) return fail(EGFEM_ERR_HIP, std::string("Krylov solve failed: ") + hipGetErrorString(e));
  const double* o = W.host_kout;
  res->status = (int)o[0];
  res->iters = (int)o[1];
  res->relres = o[2];
  res->bnorm = o[3];
  res->blocks = q.G;
  res->threads = q.NT;
  res->resident = q.resident;
  res->block_precond = q.block;
  res->overlapped = q.overlapped;
  if (res->status == EGFEM_ERR_HIP) return fail(EGFEM_ERR_HIP, "Krylov grid barrier timed out");
  return EGFEM_OK;
}

}  // namespace egfem
