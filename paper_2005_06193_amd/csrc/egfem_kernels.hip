// Tensor-action, Jacobian-emission and CSR kernels for gfx950 (FP64).
//
// The tensor kernels work on row blocks (runs of consecutive node rows that
// fit fixed LDS capacities).  One 256-thread workgroup per block:
//   stage 1  entry-parallel, fully coalesced reads of the fiber stream
//            (value + compressed index) with the pointwise coefficient
//            a_k = a0_k + u_k^2 computed from the gathered u_k (the nodal
//            update w = g(u) fused into the stream), products staged in LDS;
//   stage 2  slot-parallel fiber sums out of LDS, times the gathered u_j;
//   stage 3  row-parallel sums over the row's slots out of LDS.
// Every sum runs in a fixed order, so results are bitwise reproducible.  The
// path moves ~0.15 flop per byte and is bound by HBM bandwidth; no MFMA.
#include "egfem_internal.h"

namespace egfem {
namespace {

constexpr int kWave = 64;

// Workgroups are dispatched round-robin over the 8 XCDs of the device.  Give
// each XCD one contiguous range of row blocks so that neighbouring rows, which
// gather the same vector entries, share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblk) {
  const int64_t per = (nblk + 7) >> 3;
  const int64_t lb = (bid & 7) * per + (bid >> 3);
  return lb < nblk ? lb : -1;
}

inline unsigned xcd_grid(int64_t nblk) { return (unsigned)(((nblk + 7) >> 3) << 3); }

// Deterministic sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh4) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) sh4[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  return r;
}

// r_i = sum_{s in row i} (u_col(s) * sum_{p in A(s)} v_p a_{k_p})
//   RAW:      a given;                        out = r
//   PROBLEM:  a = a0 + w^2, w = u + alpha*delta (trial iterate when delta != 0);
//             out = F = r + K w - load, Dirichlet rows 0; partial[b] = sum F_i^2;
//             uout (optional) = w.
template <bool PROBLEM>
__global__ __launch_bounds__(kBlockThreads) void k_action(
    const int32_t* __restrict__ blk_row, int64_t nblk, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const int32_t* __restrict__ kptr,
    const int32_t* __restrict__ kidx, const double* __restrict__ val, const double* __restrict__ u,
    const double* __restrict__ delta, double alpha, const double* __restrict__ a, double a0c,
    const double* __restrict__ load, const uint8_t* __restrict__ dir,
    const double* __restrict__ kval, double* __restrict__ out, double* __restrict__ uout,
    double* __restrict__ partial) {
  __shared__ double t_lds[kCapNnz];
  __shared__ double y_lds[kCapSlots];
  __shared__ double sh4[4];
  const int64_t b = xcd_block(blockIdx.x, nblk);
  if (b < 0) return;
  const int tid = threadIdx.x;
  const int r0 = blk_row[b], r1 = blk_row[b + 1];
  const int s0 = rowptr[r0], s1 = rowptr[r1];
  const int p0 = kptr[s0], p1 = kptr[s1];

  for (int p = p0 + tid; p < p1; p += kBlockThreads) {
    const int k = kidx[p];
    double ak;
    if (PROBLEM) {
      double wk = u[k];
      if (delta) wk = fma(alpha, delta[k], wk);
      ak = fma(wk, wk, a ? a[k] : a0c);
    } else {
      ak = a[k];
    }
    t_lds[p - p0] = val[p] * ak;
  }
  __syncthreads();
  for (int s = s0 + tid; s < s1; s += kBlockThreads) {
    const int q0 = kptr[s] - p0, q1 = kptr[s + 1] - p0;
    double q = 0.0;
    for (int t = q0; t < q1; ++t) q += t_lds[t];
    const int j = col[s];
    double wj = u[j];
    if (PROBLEM) {
      if (delta) wj = fma(alpha, delta[j], wj);
      if (kval) q += kval[s];
    }
    y_lds[s - s0] = q * wj;
  }
  __syncthreads();
  double sq = 0.0;
  for (int i = r0 + tid; i < r1; i += kBlockThreads) {
    const int q0 = rowptr[i] - s0, q1 = rowptr[i + 1] - s0;
    double acc = 0.0;
    for (int t = q0; t < q1; ++t) acc += y_lds[t];
    if (PROBLEM) {
      if (load) acc -= load[i];
      const bool d = dir && dir[i];
      if (d) acc = 0.0;
      if (uout) {
        double wi = u[i];
        if (delta) wi = fma(alpha, delta[i], wi);
        uout[i] = d ? 0.0 : wi;
      }
      sq = fma(acc, acc, sq);
    }
    out[i] = acc;
  }
  if (PROBLEM && partial) {
    const double tot = block_sum256(sq, sh4);
    if (tid == 0) partial[b] = tot;
  }
}

// J_s = [K_s] + sum_{p in A(s)} v_p a_{k_p} + g_j * sum_{p in B(s)} v_p u_{j_p},
// s = (i, j); g_j = dadu[j] or 2 u_j.  Dirichlet rows -> identity rows,
// Dirichlet columns -> 0.  dinv[i] = 1 / J_ii.
__global__ __launch_bounds__(kBlockThreads) void k_jacobian(
    const int32_t* __restrict__ blk_row, int64_t nblk, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const int32_t* __restrict__ kptrA,
    const int32_t* __restrict__ kA, const double* __restrict__ vA,
    const int32_t* __restrict__ jptrB, const int32_t* __restrict__ jB,
    const double* __restrict__ vB, int sym, const double* __restrict__ u,
    const double* __restrict__ a, const double* __restrict__ a0, double a0c, int problem_a,
    const double* __restrict__ dadu, int dadu_2u, const double* __restrict__ kval,
    const uint8_t* __restrict__ dir, double* __restrict__ jval, double* __restrict__ dinv) {
  __shared__ double tA[kCapNnz];
  __shared__ double tB[kCapNnz];
  __shared__ double y[kCapSlots];
  __shared__ int scol[kCapSlots];
  __shared__ int spa[kCapSlots + 1];
  __shared__ int spb[kCapSlots + 1];
  const int64_t b = xcd_block(blockIdx.x, nblk);
  if (b < 0) return;
  const int tid = threadIdx.x;
  const int r0 = blk_row[b], r1 = blk_row[b + 1];
  const int s0 = rowptr[r0], s1 = rowptr[r1];
  const int pa0 = kptrA[s0], pa1 = kptrA[s1];
  const int pb0 = jptrB[s0], pb1 = jptrB[s1];
  const bool second = dadu || dadu_2u;

  for (int p = pa0 + tid; p < pa1; p += kBlockThreads) {
    const int k = kA[p];
    const double uk = u[k];
    const double ak = problem_a ? fma(uk, uk, a0 ? a0[k] : a0c) : a[k];
    const double v = vA[p];
    tA[p - pa0] = v * ak;
    if (sym && second) tB[p - pa0] = v * uk;
  }
  if (!sym && second)
    for (int p = pb0 + tid; p < pb1; p += kBlockThreads) tB[p - pb0] = vB[p] * u[jB[p]];
  for (int s = s0 + tid; s <= s1; s += kBlockThreads) {
    spa[s - s0] = kptrA[s] - pa0;
    spb[s - s0] = jptrB[s] - pb0;
    if (s < s1) {
      scol[s - s0] = col[s];
      y[s - s0] = kval ? kval[s] : 0.0;
    }
  }
  __syncthreads();
  for (int i = r0 + tid; i < r1; i += kBlockThreads) {
    const bool drow = dir && dir[i];
    for (int s = rowptr[i] - s0; s < rowptr[i + 1] - s0; ++s) {
      const int j = scol[s];
      double J;
      if (drow) {
        J = (j == i) ? 1.0 : 0.0;
      } else if (dir && dir[j]) {
        J = 0.0;
      } else {
        double qa = 0.0;
        for (int t = spa[s]; t < spa[s + 1]; ++t) qa += tA[t];
        J = y[s] + qa;
        if (second) {
          double qb = 0.0;
          for (int t = spb[s]; t < spb[s + 1]; ++t) qb += tB[t];
          const double g = dadu ? dadu[j] : 2.0 * u[j];
          J = fma(g, qb, J);
        }
      }
      y[s] = J;
      if (j == i && dinv) dinv[i] = 1.0 / J;
    }
  }
  __syncthreads();
  for (int s = s0 + tid; s < s1; s += kBlockThreads) jval[s] = y[s - s0];
}

// q_s = sum_{p in B(s)} v_p u_{j_p}  ((T ._2 u) in slot layout), thread per slot.
__global__ __launch_bounds__(kBlockThreads) void k_slot_mode2(int64_t slots,
                                                              const int32_t* __restrict__ jptrB,
                                                              const int32_t* __restrict__ jB,
                                                              const double* __restrict__ vB,
                                                              const double* __restrict__ u,
                                                              double* __restrict__ q) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= slots) return;
  double acc = 0.0;
  for (int p = jptrB[s]; p < jptrB[s + 1]; ++p) acc += vB[p] * u[jB[p]];
  q[s] = acc;
}

// y_i = sum_{s in row i} vals[s] x[col[s]] with L lanes per row.
template <int L>
__global__ __launch_bounds__(kBlockThreads) void k_csr_matvec(int64_t n, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ vals,
                                                              const int32_t* __restrict__ perm,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ y) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid / L;
  const int lane = (int)(gid % L);
  double acc = 0.0;
  if (row < n) {
    for (int s = rowptr[row] + lane; s < rowptr[row + 1]; s += L) {
      const double a = perm ? vals[perm[s]] : vals[s];
      acc = fma(a, x[col[s]], acc);
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
  if (row < n && lane == 0) y[row] = acc;
}

__global__ void k_permute(int64_t slots, const int32_t* __restrict__ perm,
                          const double* __restrict__ in, double* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < slots) out[s] = in[perm[s]];
}

__global__ void k_fill(double* x, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_fill_u32(unsigned* x, unsigned v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_mask_zero(double* x, const uint8_t* dir, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && dir[i]) x[i] = 0.0;
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_scale(double* x, double s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= s;
}

inline unsigned grid1d(int64_t n, int bs = kBlockThreads) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_action_raw(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_action<false>, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                     T->blk_row, T->row_blocks, T->rowptr, T->col, T->kptrA, T->kA, T->vA, u,
                     nullptr, 0.0, a, 0.0, nullptr, nullptr, nullptr, r, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_action_problem(const egfem_tensor_s* T, const ProblemView& pv, const double* u,
                                 const double* delta, double alpha, double* uout, double* F,
                                 double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_action<true>, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                     T->blk_row, T->row_blocks, T->rowptr, T->col, T->kptrA, T->kA, T->vA, u, delta,
                     alpha, pv.a0, pv.a0c, pv.load, pv.dir, pv.addK ? T->kval : nullptr, F, uout,
                     partial);
  return hipGetLastError();
}

hipError_t launch_jacobian(const egfem_tensor_s* T, const double* u, const double* a,
                           const double* a0, double a0c, int use_problem_a, const double* dadu,
                           int dadu_2u, int addK, const uint8_t* dir, double* jval, double* dinv,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_jacobian, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                     T->blk_row, T->row_blocks, T->rowptr, T->col, T->kptrA, T->kA, T->vA, T->jptrB,
                     T->jB, T->vB, T->symmetric, u, a, a0, a0c, use_problem_a, dadu, dadu_2u,
                     addK ? T->kval : nullptr, dir, jval, dinv);
  return hipGetLastError();
}

hipError_t launch_slot_mode2(const egfem_tensor_s* T, const double* u, double* q, hipStream_t st) {
  hipLaunchKernelGGL(k_slot_mode2, dim3(grid1d(T->slots)), dim3(kBlockThreads), 0, st, T->slots,
                     T->jptrB, T->jB, T->vB, u, q);
  return hipGetLastError();
}

template <int L>
static void matvec_L(const egfem_tensor_s* T, const double* vals, const int32_t* perm,
                     const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_csr_matvec<L>, dim3(grid1d(T->n * L)), dim3(kBlockThreads), 0, st, T->n,
                     T->rowptr, T->col, vals, perm, x, y);
}

static hipError_t matvec_any(const egfem_tensor_s* T, const double* vals, const int32_t* perm,
                             const double* x, double* y, hipStream_t st) {
  switch (T->lanes_per_row) {
    case 4: matvec_L<4>(T, vals, perm, x, y, st); break;
    case 8: matvec_L<8>(T, vals, perm, x, y, st); break;
    case 16: matvec_L<16>(T, vals, perm, x, y, st); break;
    case 32: matvec_L<32>(T, vals, perm, x, y, st); break;
    default: matvec_L<64>(T, vals, perm, x, y, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_csr_matvec(const egfem_tensor_s* T, const double* vals, const double* x, double* y,
                             hipStream_t st) {
  return matvec_any(T, vals, nullptr, x, y, st);
}

hipError_t launch_csr_matvec_perm(const egfem_tensor_s* T, const double* vals, const double* w,
                                  double* y, hipStream_t st) {
  return matvec_any(T, vals, T->tperm, w, y, st);
}

hipError_t launch_permute_slots(const egfem_tensor_s* T, const double* in, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_permute, dim3(grid1d(T->slots)), dim3(kBlockThreads), 0, st, T->slots,
                     T->tperm, in, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, x, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* x, unsigned v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, x, v, n);
  return hipGetLastError();
}

hipError_t launch_mask_zero(double* x, const uint8_t* dir, int64_t n, hipStream_t st) {
  if (!dir || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_zero, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, x, dir, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_scale(double* x, double s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, x, s, n);
  return hipGetLastError();
}

}  // namespace egfem
