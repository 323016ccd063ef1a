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
#include <algorithm>

#include "egfem_device.h"

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

}  // namespace

dev::TensorView view_of(const egfem_tensor_s* T) {
  dev::TensorView v;
  v.n = T->n;
  v.nblk = T->row_blocks;
  v.sym = T->symmetric;
  v.blk_row = T->blk_row;
  v.meta = reinterpret_cast<const int4*>(T->blk_meta);
  v.rowptr = T->rowptr;
  v.col = T->col;
  v.kptrA = T->kptrA;
  v.kA = T->kA;
  v.vA = T->vA;
  v.jptrB = T->jptrB;
  v.jB = T->jB;
  v.vB = T->vB;
  v.kS = T->kS;
  v.bS = T->bS;
  v.kpS = T->kpS;
  v.jpS = T->jpS;
  v.kval = T->kval;
  v.wmeta = reinterpret_cast<const int2*>(T->wmeta);
  v.wrowptr = T->wrowptr;
  v.wcol = T->wcol;
  v.wpq = T->wpq;
  v.wpq2 = T->wpq2;
  v.wqi = T->wqi;
  v.qlam = T->qlam;
  v.kSH = T->kSH;
  v.vH = T->vH;
  v.kpSH = T->kpSH;
  v.hmeta = reinterpret_cast<const int2*>(T->hmeta);
  return v;
}

namespace {

// Residual action (see action_compute), each workgroup over a contiguous run
// of row blocks, software-pipelined; XCD-aware run order:
//   RAW:      out = T:(u (x) a)
//   PROBLEM:  out = F = [K w] + T:(w (x) (a0 + w^2)) - load, w = u + alpha delta,
//             Dirichlet rows 0; partial[wg] = sum F_i^2; uout (optional) = w.
template <bool PROBLEM, bool PIPE>
__global__ __launch_bounds__(kBlockThreads) void k_action(dev::TensorView T, int64_t nrun,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ delta, double alpha,
                                                          const double* __restrict__ a, double a0c,
                                                          const double* __restrict__ load,
                                                          const uint8_t* __restrict__ dir,
                                                          const double* __restrict__ kval,
                                                          double* __restrict__ out,
                                                          double* __restrict__ uout,
                                                          double* __restrict__ partial) {
  __shared__ dev::ActionLds L;
  __shared__ double sh4[4];
  const int64_t w = xcd_block(blockIdx.x, nrun);
  if (w < 0) return;
  const int64_t b0 = T.nblk * w / nrun, b1 = T.nblk * (w + 1) / nrun;
  double sq = 0.0;
  if (PIPE)
    dev::rowblocks_action_pipelined<kBlockThreads, PROBLEM, false>(T, b0, b1, u, delta, alpha, a, a0c, load,
                                                                   dir, kval, out, uout, sq, L);
  else
    dev::rowblocks_action<kBlockThreads, PROBLEM, false>(T, b0, b1, u, delta, alpha, a, a0c, load, dir, kval,
                                                         out, uout, sq, L);
  if (PROBLEM && partial) {
    const double tot = block_sum256(sq, sh4);
    if (threadIdx.x == 0) partial[w] = tot;
  }
}

// Jacobian emission over one row block per workgroup (see rowblock_jacobian).
__global__ __launch_bounds__(kBlockThreads) void k_jacobian(dev::TensorView T, const double* __restrict__ u,
                                                            const double* __restrict__ a,
                                                            const double* __restrict__ a0, double a0c,
                                                            int problem_a, const double* __restrict__ dadu,
                                                            int dadu_2u, const double* __restrict__ kval,
                                                            const uint8_t* __restrict__ dir,
                                                            double* __restrict__ jval,
                                                            double* __restrict__ dinv) {
  __shared__ dev::JacobianLds L;
  const int64_t b = xcd_block(blockIdx.x, T.nblk);
  if (b < 0) return;
  dev::rowblock_jacobian<kBlockThreads, false>(T, b, u, a, a0, a0c, problem_a, dadu, dadu_2u, kval, dir,
                                               jval, dinv, L);
}

// W_h = P2 tensor action and Jacobian emission, one row block per workgroup
// (see rowblock_action_w2 / rowblock_jacobian_w2); partial[b] = sum F_i^2.
template <bool PROBLEM, int WK>
__global__ __launch_bounds__(kBlockThreads) void k_action_w2(dev::TensorView T, const double* __restrict__ u,
                                                             const double* __restrict__ delta, double alpha,
                                                             const double* __restrict__ a, double a0c,
                                                             const double* __restrict__ load,
                                                             const uint8_t* __restrict__ dir,
                                                             const double* __restrict__ kval,
                                                             double* __restrict__ out, double* __restrict__ uout,
                                                             double* __restrict__ partial) {
  __shared__ dev::ActionLdsW L;
  __shared__ double sh4[4];
  const int64_t b = xcd_block(blockIdx.x, T.nblk);
  if (b < 0) return;
  double sq = 0.0;
  dev::rowblock_action_w2<kBlockThreads, PROBLEM, WK>(T, b, u, delta, alpha, a, a0c, load, dir, kval, out, uout,
                                                      sq, L);
  if (PROBLEM && partial) {
    const double tot = block_sum256(sq, sh4);
    if (threadIdx.x == 0) partial[b] = tot;
  }
}

// Tensor action from the symmetric half stream, one row block per workgroup.
template <bool PROBLEM>
__global__ __launch_bounds__(kBlockThreads) void k_action_half(dev::TensorView T, const double* __restrict__ u,
                                                               const double* __restrict__ delta, double alpha,
                                                               const double* __restrict__ a, double a0c,
                                                               const double* __restrict__ load,
                                                               const uint8_t* __restrict__ dir,
                                                               const double* __restrict__ kval,
                                                               double* __restrict__ out,
                                                               double* __restrict__ uout,
                                                               double* __restrict__ partial) {
  __shared__ dev::ActionLdsH L;
  __shared__ double sh4[4];
  const int64_t b = xcd_block(blockIdx.x, T.nblk);
  if (b < 0) return;
  double sq = 0.0;
  dev::rowblock_action_half<kBlockThreads, PROBLEM>(T, b, u, delta, alpha, a, a0c, load, dir, kval, out, uout, sq,
                                                    L);
  if (PROBLEM && partial) {
    const double tot = block_sum256(sq, sh4);
    if (threadIdx.x == 0) partial[b] = tot;
  }
}

template <int WK>
__global__ __launch_bounds__(kBlockThreads) void k_jacobian_w2(dev::TensorView T, const double* __restrict__ u,
                                                               const double* __restrict__ a,
                                                               const double* __restrict__ a0, double a0c,
                                                               int problem_a, const double* __restrict__ dadu,
                                                               int dadu_2u, const double* __restrict__ kval,
                                                               const uint8_t* __restrict__ dir,
                                                               double* __restrict__ jval,
                                                               double* __restrict__ dinv) {
  __shared__ dev::RowBlockLdsW L;
  const int64_t b = xcd_block(blockIdx.x, T.nblk);
  if (b < 0) return;
  dev::rowblock_jacobian_w2<kBlockThreads, WK>(T, b, u, a, a0, a0c, problem_a, dadu, dadu_2u, kval, dir, jval,
                                               dinv, L);
}

// Element-factored stiffness action, L lanes per row, one incident cell per
// lane: r_i = sum_{e contains i} abar_e sum_b K^e_{a b} u_{c_b}, a = local index of i,
// abar_e = (sum_m a_{c_m}) / (d+1); K^e packed as the row-major upper triangle.
template <int D, int L>
__global__ __launch_bounds__(kBlockThreads) void k_action_elem(int64_t n, const int32_t* __restrict__ nptr,
                                                               const int32_t* __restrict__ inc,
                                                               const int4* __restrict__ cell4,
                                                               const double* __restrict__ kp, int kstride,
                                                               const double* __restrict__ u,
                                                               const double* __restrict__ a,
                                                               double* __restrict__ r) {
  constexpr int NL = D + 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid / L;
  const int lane = (int)(gid % L);
  double acc = 0.0;
  if (row < n) {
    for (int p = nptr[row] + lane; p < nptr[row + 1]; p += L) {
      const int code = inc[p];
      const int64_t e = code >> 2;
      const int la = code & 3;
      const int4 c = cell4[e];
      const int cv[4] = {c.x, c.y, c.z, c.w};
      double asum = 0.0, s = 0.0;
      const double* K = kp + e * kstride;
#pragma unroll
      for (int b = 0; b < NL; ++b) {
        asum += a[cv[b]];
        const int lo = la < b ? la : b, hi = la < b ? b : la;
        const int t = lo * NL - (lo * (lo - 1)) / 2 + (hi - lo);
        s = fma(K[t], u[cv[b]], s);
      }
      acc = fma(asum * (1.0 / NL), s, acc);
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
  if (row < n && lane == 0) r[row] = acc;
}

// Raw action through the unique storage of the fully symmetric mass tensor
// (each index multiset stored once):
//   r_i = T_iii u_i a_i + sum_{j ~ i} [T_iij (u_i a_j + u_j a_i) + T_ijj u_j a_j]
//       + sum_{faces {i,j,k}} T_ijk (u_j a_k + u_k a_j).
// L lanes per row.  The slot pass gathers u_j, a_j of the row's columns,
// adds the vertex and edge terms and stages the gathered values in LDS at
// their row-local slot; the face pass reads them back by slot.  Fixed lane
// order and a fixed butterfly: the sum is deterministic.
template <int L>
__global__ __launch_bounds__(kBlockThreads) void k_action_unique(int64_t n, int64_t foff, int stride,
                                                                 const int32_t* __restrict__ rowptr,
                                                                 const int32_t* __restrict__ col,
                                                                 const int32_t* __restrict__ sref,
                                                                 const int32_t* __restrict__ fptr,
                                                                 const int2* __restrict__ fref,
                                                                 const double* __restrict__ val,
                                                                 const double* __restrict__ u,
                                                                 const double* __restrict__ a,
                                                                 double* __restrict__ r) {
  extern __shared__ double lds_u[];   // [rows of the workgroup][2][stride]: u, then a
  constexpr int RPB = kBlockThreads / L;
  const int sub = (int)threadIdx.x / L, lane = (int)threadIdx.x % L;
  const int64_t row = (int64_t)blockIdx.x * RPB + sub;
  double* su = lds_u + (size_t)sub * 2 * stride;
  double* sa = su + stride;
  double acc = 0.0;
  if (row < n) {
    const int beg = rowptr[row], cnt = rowptr[row + 1] - beg;
    const double ui = u[row], ai = a[row];
    for (int s = lane; s < cnt; s += L) {
      const int j = col[beg + s];
      const double uj = u[j], aj = a[j];
      su[s] = uj;
      sa[s] = aj;
      if (j == row) {
        acc = fma(val[row], ui * ai, acc);
      } else {
        const int code = sref[beg + s];
        const int o = code & 1;
        const double* ev = val + n + (code - o);
        acc = fma(ev[o], fma(ui, aj, uj * ai), acc);
        acc = fma(ev[1 - o], uj * aj, acc);
      }
    }
  }
  __syncthreads();
  if (row < n) {
    for (int f = fptr[row] + lane; f < fptr[row + 1]; f += L) {
      const int2 fr = fref[f];
      const int sj = fr.y & 0xffff, sk = (int)((unsigned)fr.y >> 16);
      acc = fma(val[foff + fr.x], fma(su[sj], sa[sk], su[sk] * sa[sj]), acc);
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
  if (row < n && lane == 0) r[row] = acc;
}

// Coefficient of a gradient nonlinearity per cell (W_h = P0, the gradient
// interpolation of Sec. 3.2): z = sum_m u_{c_m} grad lambda_m, a_e = (c0 + c1 |z|^2)^q.
// With wv != null also the derivative weights of the Newton Jacobian,
// wv[4e + m] = d a_e / d u_{c_m} = 2 q c1 (c0 + c1 |z|^2)^(q-1) z . grad lambda_m (0 past d).
template <int D>
__global__ __launch_bounds__(kBlockThreads) void k_grad_coef(int64_t ncell, const int4* __restrict__ cell4,
                                                             const double* __restrict__ grad,
                                                             const double* __restrict__ u, double c0, double c1,
                                                             double q, int linear, double* __restrict__ a,
                                                             double* __restrict__ wv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  if (linear) {
    a[e] = 1.0;
    if (wv)
      for (int m = 0; m < 4; ++m) wv[4 * e + m] = 0.0;
    return;
  }
  const int4 c = cell4[e];
  const int cv[4] = {c.x, c.y, c.z, c.w};
  const double* G = grad + 12 * e;
  double z[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m <= D; ++m) {
    const double um = u[cv[m]];
#pragma unroll
    for (int r = 0; r < D; ++r) z[r] = fma(um, G[3 * m + r], z[r]);
  }
  double s2 = 0.0;
#pragma unroll
  for (int r = 0; r < D; ++r) s2 = fma(z[r], z[r], s2);
  const double base = fma(c1, s2, c0);
  a[e] = pow(base, q);
  if (wv) {
    const double ap = 2.0 * q * c1 * pow(base, q - 1.0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double zg = 0.0;
      if (m <= D) {
#pragma unroll
        for (int r = 0; r < D; ++r) zg = fma(z[r], G[3 * m + r], zg);
      }
      wv[4 * e + m] = m <= D ? ap * zg : 0.0;
    }
  }
}

// F_i = dir_i ? 0 : F_i - b_i, and per-workgroup partial sums of F_i^2 (grid-stride).
__global__ __launch_bounds__(kBlockThreads) void k_sub_mask_norm(int64_t n, double* __restrict__ F,
                                                                 const double* __restrict__ b,
                                                                 const uint8_t* __restrict__ dir,
                                                                 double* __restrict__ partial) {
  __shared__ double sh4[4];
  double ss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlockThreads) {
    const double f = (dir && dir[i]) ? 0.0 : F[i] - b[i];
    F[i] = f;
    ss = fma(f, f, ss);
  }
  const double tot = block_sum256(ss, sh4);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_p2_square(int64_t n, int64_t nw, const int32_t* __restrict__ edges, const double* __restrict__ u,
                            double* __restrict__ f) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nw) return;
  double v;
  if (k < n) {
    v = u[k];
  } else {
    const int64_t t = k - n;
    v = 0.5 * (u[edges[2 * t]] + u[edges[2 * t + 1]]);
  }
  f[k] = v * v;
}

// W_h = I_k: f_k = (Pi_u u)(x_k)^2 for the point k = e nq + q, Pi_u u the P1
// iterate evaluated at the point from its cell's vertices (barycentrics padded
// with zeros, vertex ids with the first).
__global__ void k_iq_square(int64_t nw, int nq, const int4* __restrict__ cell4, const double* __restrict__ qlam,
                            const double* __restrict__ u, double* __restrict__ f) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nw) return;
  const int64_t e = k / nq;
  const int q = (int)(k - e * nq);
  const int4 c = cell4[e];
  const double* lam = qlam + 4 * q;
  const double v = fma(lam[3], u[c.w], fma(lam[2], u[c.z], fma(lam[1], u[c.y], lam[0] * u[c.x])));
  f[k] = v * v;
}

__global__ void k_axpy_to(double* __restrict__ out, const double* __restrict__ x, double alpha,
                          const double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fma(alpha, y[i], x[i]);
}

// Per-workgroup partial sums of (x_i - u_i)^2 and x_i^2 (grid-stride rows):
// partial[2 g], partial[2 g + 1].
__global__ __launch_bounds__(kBlockThreads) void k_diff_norms(int64_t n, const double* __restrict__ x,
                                                              const double* __restrict__ u,
                                                              double* __restrict__ partial) {
  __shared__ double sh4[4];
  double dd = 0.0, xx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlockThreads) {
    const double xi = x[i], di = xi - u[i];
    dd = fma(di, di, dd);
    xx = fma(xi, xi, xx);
  }
  const double a = block_sum256(dd, sh4);
  const double b = block_sum256(xx, sh4);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = b;
  }
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

// Matrix of a linear time step in T's pattern, thread per row:
//   vals_s = cm M_s + ck K_s, Dirichlet rows identity, Dirichlet columns 0,
//   dinv_i = 1 / vals_(i,i).
__global__ __launch_bounds__(kBlockThreads) void k_mk_combine(int64_t n, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ mval,
                                                              const double* __restrict__ kval, double cm,
                                                              double ck, const uint8_t* __restrict__ dir,
                                                              double* __restrict__ vals,
                                                              double* __restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool di = dir && dir[i];
  double d = 1.0;
  for (int s = rowptr[i]; s < rowptr[i + 1]; ++s) {
    const int32_t j = col[s];
    double v = fma(cm, mval[s], ck * kval[s]);
    if (di) v = (j == i) ? 1.0 : 0.0;
    else if (dir && dir[j]) v = 0.0;
    vals[s] = v;
    if (j == i) d = v;
  }
  dinv[i] = 1.0 / d;
}

// Right-hand side of a semi-implicit Burgers step (Sec. 5.2), L lanes per row:
//   rhs_i = sum_{s in row i} M_s (u_j + dt src_j) + h C_i,   h = dt / 2,
//   C_i = sum_s Nf_s u_j^2 (GROUP, Nf in slot layout) or conv_i (tensor action),
//   0 on Dirichlet rows.
template <int L, bool GROUP>
__global__ __launch_bounds__(kBlockThreads) void k_burgers_rhs(int64_t n, const int32_t* __restrict__ rowptr,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ mval,
                                                               const double* __restrict__ cvals,
                                                               const double* __restrict__ u,
                                                               const double* __restrict__ src, double dt,
                                                               double h, const uint8_t* __restrict__ dir,
                                                               double* __restrict__ rhs) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid / L;
  const int lane = (int)(gid % L);
  double acc = 0.0, nacc = 0.0;
  if (row < n) {
    for (int s = rowptr[row] + lane; s < rowptr[row + 1]; s += L) {
      const int32_t j = col[s];
      const double uj = u[j];
      const double xj = src ? fma(dt, src[j], uj) : uj;
      acc = fma(mval[s], xj, acc);
      if (GROUP) nacc = fma(cvals[s], uj * uj, nacc);
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) {
    acc += __shfl_xor(acc, off, L);
    if (GROUP) nacc += __shfl_xor(nacc, off, L);
  }
  if (row < n && lane == 0) {
    const double c = GROUP ? nacc : cvals[row];
    rhs[row] = (dir && dir[row]) ? 0.0 : fma(h, c, acc);
  }
}

// Initial iterate of the next time step by polynomial extrapolation of the
// last iterates (order 0, 1 or 2), in place on u; the history shifts:
// h2 <- h1, h1 <- u (old).
__global__ void k_extrapolate(int64_t n, int order, double* __restrict__ u, double* __restrict__ h1,
                              double* __restrict__ h2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = u[i];
  if (order >= 1) {
    const double p1 = h1[i];
    u[i] = order == 2 ? fma(3.0, t - p1, h2[i]) : 2.0 * t - p1;
    h2[i] = p1;
  }
  h1[i] = t;
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

// Number of block runs (workgroups) of the action kernel: the handle's
// tuned target (0 = one block per workgroup), at least one block per run.
static bool use_half(const egfem_tensor_s* T) { return T->action_half && T->vH; }

int64_t action_runs(const egfem_tensor_s* T) {
  if (T->w2 || use_half(T)) return std::max<int64_t>(1, T->row_blocks);
  const int64_t target = T->action_runs_target > 0 ? (int64_t)T->action_runs_target : T->row_blocks;
  return std::max<int64_t>(1, std::min<int64_t>(T->row_blocks, target));
}

hipError_t launch_action_raw(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                             hipStream_t st) {
  if (T->w2) {
    auto kern = T->w2 == 1 ? k_action_w2<false, 1> : k_action_w2<false, 2>;
    hipLaunchKernelGGL(kern, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st, view_of(T), u, nullptr,
                       0.0, a, 0.0, nullptr, nullptr, nullptr, r, nullptr, nullptr);
    return hipGetLastError();
  }
  if (use_half(T)) {
    hipLaunchKernelGGL(k_action_half<false>, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                       view_of(T), u, nullptr, 0.0, a, 0.0, nullptr, nullptr, nullptr, r, nullptr, nullptr);
    return hipGetLastError();
  }
  const int64_t nrun = action_runs(T);
  auto kern = T->action_pipe ? k_action<false, true> : k_action<false, false>;
  hipLaunchKernelGGL(kern, dim3(xcd_grid(nrun)), dim3(kBlockThreads), 0, st, view_of(T), nrun, u, nullptr, 0.0,
                     a, 0.0, nullptr, nullptr, nullptr, r, nullptr, nullptr);
  return hipGetLastError();
}

template <int D, int L>
static void elem_launch(const egfem_tensor_s* T, const double* u, const double* a, double* r, hipStream_t st) {
  hipLaunchKernelGGL((k_action_elem<D, L>), dim3(grid1d(T->n * L)), dim3(kBlockThreads), 0, st, T->n, T->e_nptr,
                     T->e_inc, T->e_cell4, T->e_kp, T->e_kstride, u, a, r);
}

template <int D>
static void elem_launch_l(const egfem_tensor_s* T, const double* u, const double* a, double* r, hipStream_t st) {
  switch (T->e_lanes) {
    case 2: elem_launch<D, 2>(T, u, a, r, st); break;
    case 4: elem_launch<D, 4>(T, u, a, r, st); break;
    case 8: elem_launch<D, 8>(T, u, a, r, st); break;
    case 16: elem_launch<D, 16>(T, u, a, r, st); break;
    case 32: elem_launch<D, 32>(T, u, a, r, st); break;
    default: elem_launch<D, 64>(T, u, a, r, st); break;
  }
}

template <int L>
static void unique_launch(const egfem_tensor_s* T, const double* u, const double* a, double* r, hipStream_t st) {
  constexpr int RPB = kBlockThreads / L;
  const int64_t blocks = (T->n + RPB - 1) / RPB;
  const size_t lds = (size_t)RPB * 2 * T->u_stride * sizeof(double);
  hipLaunchKernelGGL((k_action_unique<L>), dim3(blocks), dim3(kBlockThreads), lds, st, T->n, T->u_foff,
                     T->u_stride, T->rowptr, T->col, T->u_sref, T->u_fptr, T->u_fref, T->u_val, u, a, r);
}

hipError_t launch_action_unique(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                                hipStream_t st) {
  if (T->n <= 0) return hipSuccess;
  switch (T->u_lanes) {
    case 2: unique_launch<2>(T, u, a, r, st); break;
    case 4: unique_launch<4>(T, u, a, r, st); break;
    case 8: unique_launch<8>(T, u, a, r, st); break;
    case 16: unique_launch<16>(T, u, a, r, st); break;
    case 32: unique_launch<32>(T, u, a, r, st); break;
    default: unique_launch<64>(T, u, a, r, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_grad_coef(const egfem_tensor_s* T, const double* u, double c0, double c1, double q, int linear,
                            double* a, double* wv, hipStream_t st) {
  const int64_t E = T->n_cells;
  auto kern = T->dim == 1 ? k_grad_coef<1> : (T->dim == 2 ? k_grad_coef<2> : k_grad_coef<3>);
  hipLaunchKernelGGL(kern, dim3(grid1d(E)), dim3(kBlockThreads), 0, st, E, T->e_cell4, T->e_grad, u, c0, c1, q,
                     linear, a, wv);
  return hipGetLastError();
}

hipError_t launch_jacobian_grad(const egfem_tensor_s* T, const double* a, const double* u, const double* wv,
                                const uint8_t* dir, double* jval, double* dinv, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobian_w2<3>, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st, view_of(T), u, a,
                     nullptr, 0.0, 0, wv, 0, nullptr, dir, jval, dinv);
  return hipGetLastError();
}

int launch_sub_mask_norm(int64_t n, double* F, const double* b, const uint8_t* dir, double* partial, hipStream_t st,
                         hipError_t* err) {
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlockThreads - 1) / kBlockThreads, 256));
  hipLaunchKernelGGL(k_sub_mask_norm, dim3(G), dim3(kBlockThreads), 0, st, n, F, b, dir, partial);
  *err = hipGetLastError();
  return G;
}

hipError_t launch_p2_square(const egfem_tensor_s* T, const double* u, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_p2_square, dim3(grid1d(T->n_w)), dim3(kBlockThreads), 0, st, T->n, T->n_w, T->p2_edges, u,
                     f);
  return hipGetLastError();
}

hipError_t launch_iq_square(const egfem_tensor_s* T, const double* u, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_iq_square, dim3(grid1d(T->n_w)), dim3(kBlockThreads), 0, st, T->n_w, T->nq, T->e_cell4,
                     T->qlam, u, f);
  return hipGetLastError();
}

hipError_t launch_axpy(double* out, const double* x, double alpha, const double* y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_to, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, out, x, alpha, y, n);
  return hipGetLastError();
}

hipError_t launch_action_elementwise(const egfem_tensor_s* T, const double* u, const double* a, double* r,
                                     hipStream_t st) {
  switch (T->dim) {
    case 1: elem_launch_l<1>(T, u, a, r, st); break;
    case 2: elem_launch_l<2>(T, u, a, r, st); break;
    default: elem_launch_l<3>(T, u, a, r, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_action_problem(const egfem_tensor_s* T, const ProblemView& pv, const double* u,
                                 const double* delta, double alpha, double* uout, double* F,
                                 double* partial, hipStream_t st) {
  if (T->w2) {
    auto kern = T->w2 == 1 ? k_action_w2<true, 1> : k_action_w2<true, 2>;
    hipLaunchKernelGGL(kern, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st, view_of(T), u, delta,
                       alpha, pv.a0, pv.a0c, pv.load, pv.dir, pv.addK ? T->kval : nullptr, F, uout, partial);
    return hipGetLastError();
  }
  if (use_half(T)) {
    hipLaunchKernelGGL(k_action_half<true>, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                       view_of(T), u, delta, alpha, pv.a0, pv.a0c, pv.load, pv.dir, pv.addK ? T->kval : nullptr,
                       F, uout, partial);
    return hipGetLastError();
  }
  const int64_t nrun = action_runs(T);
  auto kern = T->action_pipe ? k_action<true, true> : k_action<true, false>;
  hipLaunchKernelGGL(kern, dim3(xcd_grid(nrun)), dim3(kBlockThreads), 0, st, view_of(T), nrun, u, delta, alpha,
                     pv.a0, pv.a0c, pv.load, pv.dir, pv.addK ? T->kval : nullptr, F, uout, partial);
  return hipGetLastError();
}

hipError_t launch_jacobian(const egfem_tensor_s* T, const double* u, const double* a,
                           const double* a0, double a0c, int use_problem_a, const double* dadu,
                           int dadu_2u, int addK, const uint8_t* dir, double* jval, double* dinv,
                           hipStream_t st) {
  if (T->w2) {
    auto kern = T->w2 == 1 ? k_jacobian_w2<1> : (T->w2 == 2 ? k_jacobian_w2<2> : k_jacobian_w2<3>);
    hipLaunchKernelGGL(kern, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st, view_of(T), u, a, a0, a0c,
                       use_problem_a, dadu, dadu_2u, addK ? T->kval : nullptr, dir, jval, dinv);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_jacobian, dim3(xcd_grid(T->row_blocks)), dim3(kBlockThreads), 0, st,
                     view_of(T), u, a, a0, a0c, use_problem_a, dadu, dadu_2u,
                     addK ? T->kval : nullptr, dir, jval, dinv);
  return hipGetLastError();
}

int launch_diff_norms(int64_t n, const double* x, const double* u, double* partial, hipStream_t st,
                      hipError_t* err) {
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlockThreads - 1) / kBlockThreads, 256));
  hipLaunchKernelGGL(k_diff_norms, dim3(G), dim3(kBlockThreads), 0, st, n, x, u, partial);
  *err = hipGetLastError();
  return G;
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

hipError_t launch_mk_combine(const egfem_tensor_s* T, double cm, double ck, const uint8_t* dir, double* vals,
                             double* dinv, hipStream_t st) {
  hipLaunchKernelGGL(k_mk_combine, dim3(grid1d(T->n)), dim3(kBlockThreads), 0, st, T->n, T->rowptr, T->col,
                     T->mval, T->kval, cm, ck, dir, vals, dinv);
  return hipGetLastError();
}

template <int L>
static void burgers_rhs_L(const egfem_tensor_s* T, bool group, const double* u, const double* src, double dt,
                          const double* cvals, const uint8_t* dir, double* rhs, hipStream_t st) {
  auto kern = group ? k_burgers_rhs<L, true> : k_burgers_rhs<L, false>;
  hipLaunchKernelGGL(kern, dim3(grid1d(T->n * L)), dim3(kBlockThreads), 0, st, T->n, T->rowptr, T->col, T->mval,
                     cvals, u, src, dt, 0.5 * dt, dir, rhs);
}

hipError_t launch_burgers_rhs(const egfem_tensor_s* T, bool group, const double* u, const double* src, double dt,
                              const double* cvals, const uint8_t* dir, double* rhs, hipStream_t st) {
  switch (T->lanes_per_row) {
    case 4: burgers_rhs_L<4>(T, group, u, src, dt, cvals, dir, rhs, st); break;
    case 8: burgers_rhs_L<8>(T, group, u, src, dt, cvals, dir, rhs, st); break;
    case 16: burgers_rhs_L<16>(T, group, u, src, dt, cvals, dir, rhs, st); break;
    case 32: burgers_rhs_L<32>(T, group, u, src, dt, cvals, dir, rhs, st); break;
    default: burgers_rhs_L<64>(T, group, u, src, dt, cvals, dir, rhs, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_extrapolate(int64_t n, int order, double* u, double* h1, double* h2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extrapolate, dim3(grid1d(n)), dim3(kBlockThreads), 0, st, n, order, u, h1, h2);
  return hipGetLastError();
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
