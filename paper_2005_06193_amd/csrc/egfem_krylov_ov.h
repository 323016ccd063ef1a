// BiCGStab with the block-Jacobi preconditioner, arranged so that the
// preconditioner's workgroup-local work runs while the team's reductions
// complete, and so that a product's gather of other workgroups' vector
// entries needs no separate synchronisation.
//
// Reductions are split into an arrival (store this workgroup's partials) and
// a wait (read the totals that one aggregating workgroup forms from all
// partials in rank order, so every workgroup obtains bitwise the same
// totals); the Chebyshev steps of the preconditioner run in between.  Both
// exchanges carry completion flags (below), so an arrival is a plain store.
//
// Entries of other workgroups' rows ("ghosts": the out-of-part columns of a
// part's rows) are kept in LDS next to the part's own values, so every
// product reads LDS only.  A ghost's values follow from two vectors its owner
// publishes per iteration, vh and q = zh - alpha yh, and the iteration's
// scalars: the ghost's thread repeats the owner's recurrences operation by
// operation (same fma sequence, same operands), so its copies of phat and rh
// are bitwise the owner's.  Both vectors are published inside a reduction's
// window and loaded while the reduction completes, so a product never waits
// for a separate exchange.  Published entries carry completion flags: an
// entry is stored as two 64-bit words, each holding 32 bits of the FP64 value
// and a 32-bit flag (the launch's salt and the publication number); 64-bit
// stores and loads are single-copy atomic, so a reader that sees the expected
// flag in both words has the value, and polls until it does.  The words are
// written and read with agent-scope (coherent) accesses, in a buffer only
// this kernel writes; the salt differs from every earlier launch since the
// buffer was last zeroed (at allocation and whenever the salt wraps), so
// words left from those launches never match.
// The two team reductions of an iteration keep every read of a published
// vector ahead of its next overwrite.
//
// Right-preconditioned BiCGStab (van der Vorst) with M the block-Jacobi
// operator (k Chebyshev steps on the workgroup's diagonal block: a fixed
// linear operator, no communication).  Every product with J is formed
// explicitly (v = J phat, z = J rh, y = J vh), so the recurrences of r and x
// stay consistent; only the preconditioned vectors use the linearity of M:
//   A: v = J phat, z = J rh        arrive (rhat,v) (r,r);  vh = M^-1 v, zh = M^-1 z;  publish vh;
//                                  wait -> alpha;  ghosts' vh
//   B: y = J vh; s = r - alpha v; t = z - alpha y
//                                  arrive (t,s) (t,t) (rhat,s) (rhat,t);  yh = M^-1 y;
//                                  publish q = zh - alpha yh;  wait -> omega, beta;  ghosts' q
//   C: sh = rh - alpha vh (= M^-1 s);  x += alpha phat + omega sh;  r = s - omega t;
//      rh = sh - omega q (= M^-1 r);  phat = rh + beta (phat - omega vh)   (own rows and ghosts)
#pragma once

#include "egfem_device.h"

namespace egfem {
namespace dev {

constexpr unsigned kLLEpochBits = 20;
constexpr unsigned kLLEpochMask = (1u << kLLEpochBits) - 1u;

__device__ __forceinline__ unsigned ll_flag(unsigned salt, unsigned ep) {
  return (salt << kLLEpochBits) | (ep & kLLEpochMask);
}
__device__ __forceinline__ void ll_store(uint64_t* w, double v, unsigned flag) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  __hip_atomic_store(w, ((uint64_t)flag << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, ((uint64_t)flag << 32) | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ll_load(const uint64_t* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool ll_ok(uint64_t w, unsigned flag) { return (unsigned)(w >> 32) == flag; }
__device__ __forceinline__ double ll_value(uint64_t lo, uint64_t hi) {
  return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}

// Bounded poll step of a flagged gather: returns true when the team aborted.
__device__ __forceinline__ bool ll_spin(unsigned* abort_word, unsigned& spins) {
  __builtin_amdgcn_s_sleep(1);
  if (++spins >= kSpinCap) {
    __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return (spins & 1023u) == 0 &&
         __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// Reductions through one aggregating workgroup that owns no rows (the last
// workgroup of the grid).  Every solver workgroup stores its partials of the
// kAggValues values of a reduction as flagged words (no atomics, no wait: the
// arrival is a store; values a reduction does not use are stored as 0); the
// aggregator polls all partials of reduction e, adds them in rank order and
// stores the totals as flagged words; the solver workgroups poll the totals.
// Every workgroup therefore holds bitwise the same totals.  Partials and
// totals live in a ring of two sets: a set is rewritten for reduction e + 2
// only after every solver workgroup read the totals of e + 1, which it does
// after it read those of e (the aggregator reads partials in order).  The
// aggregator leaves when workgroup 0 stores the exit word, or on an abort.
constexpr int kAggValues = 4;

struct AggRed {
  unsigned rank, size, salt;  // size: solver workgroups (the aggregator is rank size)
  uint64_t* part;             // [2][kAggValues][2][size] partial words (value halves)
  uint64_t* tot;              // [2][kAggValues][2] total words
  uint64_t* exit_word;
  unsigned* abort_word;
  unsigned epoch = 0;         // reductions started
};

// Arrival: thread contributions v[q] (q < m <= kAggValues) summed per
// workgroup and stored (every value of the set, unused ones as 0).
template <int NT>
__device__ void agg_arrive(AggRed& a, const double (&v)[kMaxRed], int m, double* sh) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < kAggValues; ++q) {
    if (q < m) {
      const double x = wave_sum(v[q]);
      if (lane == 0) sh[q * NW + wave] = x;
    }
  }
  lds_barrier();
  const unsigned e = ++a.epoch;
  uint64_t* set = a.part + (size_t)(e & 1u) * kAggValues * 2 * a.size;
  if (wave == 0 && lane < 2 * kAggValues) {
    const int q = lane >> 1, h = lane & 1;
    double acc = 0.0;
    if (q < m)
      for (int w = 0; w < NW; ++w) acc += sh[q * NW + w];
    const unsigned long long b = (unsigned long long)__double_as_longlong(acc);
    const unsigned bits = h ? (unsigned)(b >> 32) : (unsigned)(b & 0xffffffffull);
    __hip_atomic_store(set + ((size_t)q * 2 + h) * a.size + a.rank, ((uint64_t)ll_flag(a.salt, e) << 32) | bits,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait (solver workgroups) for the totals of the latest arrival.  Returns
// true when the team aborted (the same answer in every thread).
template <int NT>
__device__ bool agg_wait(AggRed& a, double (&v)[kMaxRed], int m, double* sh, int* sh_state) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const unsigned e = a.epoch;
  const unsigned flag = ll_flag(a.salt, e);
  const uint64_t* tot = a.tot + (size_t)(e & 1u) * kAggValues * 2;
  int ab = 0;
  if (wave == 0) {
    // lane 2q + h polls half h of total q
    const int qq = lane < 2 * kAggValues ? lane : 0;
    uint64_t w = 0;
    unsigned spins = 0;
    while (true) {
      w = ll_load(tot + qq);
      if (__all(ll_ok(w, flag))) break;
      if (ll_spin(a.abort_word, spins)) {
        ab = 1;
        break;
      }
    }
    const uint64_t other = (uint64_t)__shfl_xor((long long)w, 1);
    if (lane < 2 * m && (lane & 1) == 0) sh[kMaxRed * NW + (lane >> 1)] = ll_value(w, other);
    if (lane == 0) *sh_state = ab;
  }
  lds_barrier();
  const bool aborted = *sh_state != 0;
#pragma unroll
  for (int q = 0; q < kMaxRed; ++q)
    if (q < m) v[q] = sh[kMaxRed * NW + q];
  lds_barrier();   // sh is reused by the next reduction
  return aborted;
}

// The aggregator's loop (run by the workgroup of rank a.size; wave q adds
// value q, so NT / 64 >= kAggValues).  Leaves when the exit word carries
// this launch's salt, or on an abort.
template <int NT>
__device__ void agg_serve(AggRed& a) {
  static_assert(NT / kWave >= kAggValues, "one wave per value");
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const unsigned G = a.size;
  const unsigned exit_flag = ll_flag(a.salt, kLLEpochMask);
  for (unsigned e = 1;; ++e) {
    const unsigned flag = ll_flag(a.salt, e);
    int quit = 0;
    double acc = 0.0;
    if (wave < kAggValues) {
      // every partial of value `wave` polled at once (lane l: ranks l, l + 64, ...)
      const uint64_t* lo = a.part + (size_t)(e & 1u) * kAggValues * 2 * G + (size_t)wave * 2 * G;
      const uint64_t* hi = lo + G;
      constexpr int RMAX = (kMaxKrylovBlocks + kWave - 1) / kWave;
      const int R = (int)((G + kWave - 1) / kWave);
      uint64_t wl[RMAX], wh[RMAX];
      unsigned spins = 0;
      while (true) {
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
          if (r < R) {
            const unsigned idx = min((unsigned)(lane + kWave * r), G - 1);
            wl[r] = ll_load(lo + idx);
            wh[r] = ll_load(hi + idx);
          }
        }
        bool ok = true;
#pragma unroll
        for (int r = 0; r < RMAX; ++r)
          if (r < R) ok = ok && ll_ok(wl[r], flag) && ll_ok(wh[r], flag);
        if (__all(ok)) break;
        if ((unsigned)(ll_load(a.exit_word) >> 32) == exit_flag || ll_spin(a.abort_word, spins)) {
          quit = 1;
          break;
        }
      }
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
        if (r < R && (unsigned)(lane + kWave * r) < G) acc += ll_value(wl[r], wh[r]);
      if (!quit) {
        acc = wave_sum(acc);
        if (lane < 2) {
          const unsigned long long b = (unsigned long long)__double_as_longlong(acc);
          const unsigned bits = lane ? (unsigned)(b >> 32) : (unsigned)(b & 0xffffffffull);
          __hip_atomic_store(a.tot + (size_t)(e & 1u) * kAggValues * 2 + (size_t)wave * 2 + lane,
                             ((uint64_t)flag << 32) | bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    // every wave leaves together: the first quitting wave decides for all
    if (__syncthreads_or(quit)) return;
  }
}

// Kernel arguments of the overlapped BiCGStab beyond KArgs.
struct OvArgs {
  uint64_t* llv;          // [3][n][2] flagged words of the published phat (initial), vh, q
  const int16_t* kext;    // [slots] part-local position of the column (>= 0) or -1 - ghost index
  const int32_t* gptr;    // [G + 1] ghost range of every part
  const int32_t* gcol;    // [ghosts] global column of every ghost
  uint64_t* part;         // reduction partial words [2][kAggValues][2][G]
  uint64_t* tot;          // reduction total words [2][kAggValues][2]
  uint64_t* exit_word;    // set by workgroup 0 when the solve ends (releases the aggregator)
  unsigned salt;          // 1 .. 4095: differs from every launch since the words were zeroed
};

// One ghost's published entry: the two words, loaded ahead (while a
// reduction completes) and checked after.
struct GhostWords {
  uint64_t lo = 0, hi = 0;
};
__device__ __forceinline__ void ghost_load(const uint64_t* vec, unsigned gc, GhostWords& w) {
  w.lo = ll_load(vec + 2 * (size_t)gc);
  w.hi = ll_load(vec + 2 * (size_t)gc + 1);
}
// Polls until the wave's ghost words carry `flag` (the first check uses the
// words loaded ahead); returns true when the team aborted.
__device__ __forceinline__ bool ghost_wait(const uint64_t* vec, unsigned gc, unsigned flag, GhostWords& w,
                                           unsigned* abort_word) {
  unsigned spins = 0;
  while (!__all(ll_ok(w.lo, flag) && ll_ok(w.hi, flag))) {
    if (ll_spin(abort_word, spins)) return true;
    ghost_load(vec, gc, w);
  }
  return false;
}

// Workgroup-uniform "any" of p through an LDS word that is zero on entry and
// left zero (uses are separated by further workgroup barriers).
__device__ __forceinline__ bool wg_any(bool p, int* word) {
  if (p) *word = 1;
  lds_barrier();
  const bool r = *word != 0;
  lds_barrier();
  if (threadIdx.x == 0) *word = 0;
  return r;
}

// z = M_b^-1 x for NV vectors (see block_cheb), x and z of this thread's row.
template <int NT, int K, int NV>
__device__ __forceinline__ void ov_prec(const int (&li)[K], const double (&aa)[K], double ad, double d, bool own,
                                        int steps, const ChebParams& cp, double* cheb, const double (&x)[NV],
                                        double (&z)[NV]) {
  if (steps > 0) {
    block_cheb<NT, K, NV, true>(li, aa, ad, d, own, steps, cp, cheb, x, z);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) z[v] = d * x[v];
  }
}

template <int NT, int K>
__device__ KOut team_bicgstab_ov(AggRed& ar, const KArgs& A, const OvArgs& O, int rb, int re, double* sh,
                                 int* sh_state) {
  static_assert(NT / kWave >= kAggValues, "reductions carry kAggValues values");
  constexpr int LX = 2 * NT + 1;   // LDS vector: own rows [0, NT), zero at NT, ghosts from NT + 1
  __shared__ double xph[LX], xrh[LX], xvh[LX];
  __shared__ double cheb_lds[4 * (NT + 1)];
  unsigned* const abort_word = ar.abort_word;
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  const int tid = (int)threadIdx.x;
  const int i = rb + tid;
  const bool own = i < re;
  const int q = max(min(i, re - 1), 0);
  const int row = A.rlist[q];
  const int64_t n = A.n;
  // ---- the row: LDS positions of its entries (own rows, or ghosts) --------
  // px[k]: position in the LDS vectors (NT: the zero entry); li[k]: the
  // in-part off-diagonal positions only (the block operator)
  int px[K], li[K];
  double aa[K];
  const int beg = A.rowptr[row], end = A.rowptr[row + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = min(beg + k, end - 1);
    const bool real = own && beg + k < end;
    const int c = A.col[s];
    const int l = O.kext[s];
    const double w = A.val[A.perm ? A.perm[s] : s];
    px[k] = real ? (l >= 0 ? l : NT + 1 + (-1 - l)) : NT;
    li[k] = (real && l >= 0 && c != row) ? l : NT;
    aa[k] = real ? w : 0.0;
  }
  double ad = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (px[k] == tid && own) ad = aa[k];   // the diagonal (own position)
  // aa without the diagonal for the block operator
  double ab[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ab[k] = li[k] < NT ? aa[k] : 0.0;
  const double d = A.dinv[row];
  const double b = own ? A.rhs_scale * A.rhs[row] : 0.0;
  // ghosts of this part: thread t < ng keeps ghost t
  const int g0 = O.gptr[blockIdx.x], ng = O.gptr[blockIdx.x + 1] - g0;   // ng <= NT (host)
  const bool gown = tid < ng;
  const unsigned gc = (unsigned)O.gcol[g0 + min(tid, max(ng - 1, 0))];
  const bool bj = A.cheb_steps > 0;
  ChebParams cp{1.0, 1.0, 1.0};
  if (bj) {
    cp = cheb_params<NT, K>(li, ab, ad, d, cheb_lds, A.cheb_ratio);
    if (threadIdx.x < 4) cheb_lds[(threadIdx.x >> 1) * 2 * (NT + 1) + (threadIdx.x & 1) * (NT + 1) + NT] = 0.0;
  }
  if (threadIdx.x == 0) {
    xph[NT] = 0.0;
    xrh[NT] = 0.0;
    xvh[NT] = 0.0;
  }
  uint64_t* const llp = O.llv;                      // initial phat (= rh)
  uint64_t* const llv = O.llv + 2 * (size_t)n;      // vh
  uint64_t* const llq = O.llv + 4 * (size_t)n;      // q
  unsigned ep = 0;                                  // publication number (per iteration)
  auto spmv = [&](const double* xv) -> double {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fma(aa[k], xv[px[k]], acc);
    return acc;
  };
  // ---- r = b - J x0 ; rhat = r ; phat = rh = M^-1 r --------------------------
  double x = 0.0, r = b;
  if (!A.x_zero) {
    x = own ? A.x[row] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fma(aa[k], A.x[A.col[min(beg + k, end - 1)]], acc);
    if (own) r = b - acc;
  }
  double ph, rh;
  {
    const double xs[1] = {r};
    double zs[1];
    ov_prec<NT, K, 1>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
    ph = rh = own ? zs[0] : 0.0;
  }
  // initial phat = rh: own rows to LDS, published for the ghosts of other parts
  ++ep;
  xph[tid] = ph;
  xrh[tid] = rh;
  if (own) ll_store(llp + 2 * (size_t)row, ph, ll_flag(O.salt, ep));
  double gph = 0.0, grh = 0.0, gvh = 0.0;   // this thread's ghost (when gown)
  EGFEM_ZERO_RED();
  red[0] = b * b;
  agg_arrive<NT>(ar, red, 1, sh);
  {
    GhostWords w;
    if (ng > 0) ghost_load(llp, gc, w);
    const bool gab = ng > 0 && ghost_wait(llp, gc, ll_flag(O.salt, ep), w, abort_word);
    if ((o.abort = agg_wait<NT>(ar, red, 1, sh, sh_state))) return o;
    if ((o.abort = wg_any(gab, &sh_state[1]))) return o;
    if (gown) {
      gph = grh = ll_value(w.lo, w.hi);
      xph[NT + 1 + tid] = gph;
      xrh[NT + 1 + tid] = grh;
    }
    lds_barrier();
  }
  const double bnorm = sqrt(red[0]);
  o.bnorm = bnorm;
  if (bnorm == 0.0) {
    if (own) A.x[row] = 0.0;
    o.status = EGFEM_OK;
    return o;
  }
  double rho = 0.0, rnorm = 0.0, r0norm = -1.0, rhat = r;
  int restarts = 0, it = 0;
  while (true) {
    // ---- A: v = J phat, z = J rh (LDS) ----------------------------------------
    const double v = spmv(xph), z = spmv(xrh);
    EGFEM_ZERO_RED();
    if (own) {
      red[0] = rhat * v;
      red[1] = r * r;
    }
    agg_arrive<NT>(ar, red, 2, sh);
    double vh, zh;
    {
      // preconditioned v and z while the reduction completes
      const double xs[2] = {v, z};
      double zs[2];
      ov_prec<NT, K, 2>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
      vh = own ? zs[0] : 0.0;
      zh = own ? zs[1] : 0.0;
    }
    ++ep;
    const unsigned fl = ll_flag(O.salt, ep);
    xvh[tid] = vh;
    if (own) ll_store(llv + 2 * (size_t)row, vh, fl);
    GhostWords wv;
    if (ng > 0) ghost_load(llv, gc, wv);   // the ghosts' vh, while the reduction completes
    if ((o.abort = agg_wait<NT>(ar, red, 2, sh, sh_state))) break;
    {
      const bool gab = ng > 0 && ghost_wait(llv, gc, fl, wv, abort_word);
      if ((o.abort = wg_any(gab, &sh_state[1]))) break;
    }
    if (gown) {
      gvh = ll_value(wv.lo, wv.hi);
      xvh[NT + 1 + tid] = gvh;
    }
    lds_barrier();
    const double rv = red[0];
    rnorm = sqrt(red[1]);
    if (r0norm < 0.0) {
      r0norm = rnorm;
      rho = red[1];
    }
    if (!isfinite(rnorm) || !isfinite(rho)) { o.status = EGFEM_NONFINITE; break; }
    if (rnorm <= A.rtol * bnorm) { o.status = EGFEM_OK; break; }
    if (it >= A.max_iter) { o.status = EGFEM_NOT_CONVERGED; break; }
    if (fabs(rho) <= 1e-15 * r0norm * rnorm) {
      // lost bi-orthogonality: restart once from the current residual (p = r);
      // the ghosts follow (their phat becomes their rh)
      if (restarts++ >= 1) { o.status = EGFEM_BREAKDOWN; break; }
      rhat = r;
      ph = rh;
      rho = red[1];
      r0norm = rnorm;
      xph[tid] = ph;
      if (gown) {
        gph = grh;
        xph[NT + 1 + tid] = gph;
      }
      lds_barrier();
      continue;
    }
    if (rv == 0.0 || !isfinite(rv)) { o.status = isfinite(rv) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
    const double alpha = rho / rv;
    // ---- B: y = J vh ; s, t ; q = zh - alpha yh ---------------------------------
    const double y = spmv(xvh);
    const double sv = fma(-alpha, v, r);
    const double tv = fma(-alpha, y, z);
    EGFEM_ZERO_RED();
    if (own) {
      red[0] = tv * sv;
      red[1] = tv * tv;
      red[2] = rhat * sv;
      red[3] = rhat * tv;
    }
    agg_arrive<NT>(ar, red, 4, sh);
    double qv;
    {
      const double xs[1] = {y};
      double zs[1];
      ov_prec<NT, K, 1>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
      qv = own ? fma(-alpha, zs[0], zh) : 0.0;
    }
    ++ep;
    const unsigned fq = ll_flag(O.salt, ep);
    if (own) ll_store(llq + 2 * (size_t)row, qv, fq);
    GhostWords wq;
    if (ng > 0) ghost_load(llq, gc, wq);   // the ghosts' q, while the reduction completes
    if ((o.abort = agg_wait<NT>(ar, red, 4, sh, sh_state))) break;
    {
      const bool gab = ng > 0 && ghost_wait(llq, gc, fq, wq, abort_word);
      if ((o.abort = wg_any(gab, &sh_state[1]))) break;
    }
    ++it;
    if (red[1] == 0.0 || !isfinite(red[1])) {
      o.status = isfinite(red[1]) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE;
      break;
    }
    const double omega = red[0] / red[1];
    if (omega == 0.0) { o.status = EGFEM_BREAKDOWN; break; }
    const double rho_new = fma(-omega, red[3], red[2]);
    const double beta = (rho_new / rho) * (alpha / omega);
    rho = rho_new;
    // ---- C: own rows and ghosts, the same operations ----------------------------
    const double shat = fma(-alpha, vh, rh);   // M^-1 s
    x = fma(alpha, ph, fma(omega, shat, x));
    r = fma(-omega, tv, sv);
    rh = fma(-omega, qv, shat);
    ph = fma(beta, fma(-omega, vh, ph), rh);
    if (!own) {
      r = 0.0;
      rh = 0.0;
      ph = 0.0;
    }
    xph[tid] = ph;
    xrh[tid] = rh;
    if (gown) {
      const double gq = ll_value(wq.lo, wq.hi);
      const double gs = fma(-alpha, gvh, grh);
      grh = fma(-omega, gq, gs);
      gph = fma(beta, fma(-omega, gvh, gph), grh);
      xph[NT + 1 + tid] = gph;
      xrh[NT + 1 + tid] = grh;
    }
    lds_barrier();
  }
#undef EGFEM_ZERO_RED
  if (!o.abort && own) A.x[row] = x;
  o.iters = it;
  o.rnorm = rnorm;
  return o;
}

// Preconditioned conjugate gradients (Chronopoulos and Gear: one reduction
// per iteration) in the same arrangement: with u = M^-1 r and w = J u,
//   w = J u (LDS)                    arrive (r,u) (w,u) (r,r);  wh = M^-1 w;  publish wh;
//                                    wait -> alpha, beta;  ghosts' wh
//   p = u + beta p;  s = w + beta s;  x += alpha p;  r -= alpha s;
//   sh = wh + beta sh (= M^-1 s);  u -= alpha sh (= M^-1 r)   (own rows and ghosts)
// so the block operator is applied inside the reduction's window and the
// ghosts' u follows their owners' recurrences bitwise.  The recurrence for u
// drifts from M^-1 r by rounding, which matters once r is small (gamma =
// (r, u) then loses its sign): below ||r|| <= kCgExact ||r_ref|| every
// iteration forms u = M^-1 r explicitly after the reduction and publishes it
// for the ghosts.  Stops when ||r|| <= rtol ||r0|| (rel_r0) or rtol ||b||; a
// non-positive curvature or gamma reports EGFEM_BREAKDOWN.
constexpr double kCgExact = 1e-7;
template <int NT, int K>
__device__ KOut team_pcg_ov(AggRed& ar, const KArgs& A, const OvArgs& O, int rb, int re, double* sh,
                            int* sh_state) {
  static_assert(NT / kWave >= kAggValues, "reductions carry kAggValues values");
  constexpr int LX = 2 * NT + 1;
  __shared__ double xu[LX];
  __shared__ double cheb_lds[4 * (NT + 1)];
  unsigned* const abort_word = ar.abort_word;
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  const int tid = (int)threadIdx.x;
  const int i = rb + tid;
  const bool own = i < re;
  const int q = max(min(i, re - 1), 0);
  const int row = A.rlist[q];
  const int64_t n = A.n;
  int px[K], li[K];
  double aa[K];
  const int beg = A.rowptr[row], end = A.rowptr[row + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = min(beg + k, end - 1);
    const bool real = own && beg + k < end;
    const int c = A.col[s];
    const int l = O.kext[s];
    px[k] = real ? (l >= 0 ? l : NT + 1 + (-1 - l)) : NT;
    li[k] = (real && l >= 0 && c != row) ? l : NT;
    aa[k] = real ? A.val[s] : 0.0;
  }
  double ad = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (px[k] == tid && own) ad = aa[k];
  double ab[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ab[k] = li[k] < NT ? aa[k] : 0.0;
  const double d = A.dinv[row];
  const double b = own ? A.rhs_scale * A.rhs[row] : 0.0;
  const int g0 = O.gptr[blockIdx.x], ng = O.gptr[blockIdx.x + 1] - g0;
  const bool gown = tid < ng;
  const unsigned gc = (unsigned)O.gcol[g0 + min(tid, max(ng - 1, 0))];
  const bool bj = A.cheb_steps > 0;
  ChebParams cp{1.0, 1.0, 1.0};
  if (bj) {
    cp = cheb_params<NT, K>(li, ab, ad, d, cheb_lds, A.cheb_ratio);
    if (threadIdx.x < 4) cheb_lds[(threadIdx.x >> 1) * 2 * (NT + 1) + (threadIdx.x & 1) * (NT + 1) + NT] = 0.0;
  }
  if (threadIdx.x == 0) xu[NT] = 0.0;
  uint64_t* const llu = O.llv;                      // initial u
  uint64_t* const llw = O.llv + 2 * (size_t)n;      // wh
  unsigned ep = 0;
  double x = 0.0, r = b;
  if (!A.x_zero) {
    x = own ? A.x[row] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fma(aa[k], A.x[A.col[min(beg + k, end - 1)]], acc);
    if (own) r = b - acc;
  }
  double u;
  {
    const double xs[1] = {r};
    double zs[1];
    ov_prec<NT, K, 1>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
    u = own ? zs[0] : 0.0;
  }
  ++ep;
  xu[tid] = u;
  if (own) ll_store(llu + 2 * (size_t)row, u, ll_flag(O.salt, ep));
  double gu = 0.0, gs = 0.0;   // this thread's ghost: u and sh
  EGFEM_ZERO_RED();
  red[0] = b * b;
  agg_arrive<NT>(ar, red, 1, sh);
  {
    GhostWords w;
    if (ng > 0) ghost_load(llu, gc, w);
    const bool gab = ng > 0 && ghost_wait(llu, gc, ll_flag(O.salt, ep), w, abort_word);
    if ((o.abort = agg_wait<NT>(ar, red, 1, sh, sh_state))) return o;
    if ((o.abort = wg_any(gab, &sh_state[1]))) return o;
    if (gown) {
      gu = ll_value(w.lo, w.hi);
      xu[NT + 1 + tid] = gu;
    }
    lds_barrier();
  }
  const double bnorm = sqrt(red[0]);
  double ref = bnorm, gamma_prev = 0.0, alpha_prev = 0.0, rnorm = 0.0;
  double p = 0.0, sv = 0.0, shv = 0.0;
  int it = 0;
  bool exact = false;   // u = M^-1 r formed explicitly (uniform over the team)
  while (true) {
    double wv = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) wv = fma(aa[k], xu[px[k]], wv);
    EGFEM_ZERO_RED();
    if (own) {
      red[0] = r * u;
      red[1] = wv * u;
      red[2] = r * r;
    }
    agg_arrive<NT>(ar, red, 3, sh);
    double wh = 0.0;
    GhostWords ww;
    unsigned fw = 0;
    if (!exact) {
      const double xs[1] = {wv};
      double zs[1];
      ov_prec<NT, K, 1>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
      wh = own ? zs[0] : 0.0;
      ++ep;
      fw = ll_flag(O.salt, ep);
      if (own) ll_store(llw + 2 * (size_t)row, wh, fw);
      if (ng > 0) ghost_load(llw, gc, ww);
    }
    if ((o.abort = agg_wait<NT>(ar, red, 3, sh, sh_state))) break;
    if (!exact) {
      const bool gab = ng > 0 && ghost_wait(llw, gc, fw, ww, abort_word);
      if ((o.abort = wg_any(gab, &sh_state[1]))) break;
    }
    const double gamma = red[0], delta = red[1];
    rnorm = sqrt(red[2]);
    if (it == 0 && A.rel_r0) ref = rnorm;
    if (!isfinite(rnorm) || !isfinite(gamma) || !isfinite(delta)) { o.status = EGFEM_NONFINITE; break; }
    if (rnorm <= A.rtol * ref) { o.status = EGFEM_OK; break; }
    if (it >= A.max_iter) { o.status = EGFEM_NOT_CONVERGED; break; }
    const double beta = it == 0 ? 0.0 : gamma / gamma_prev;
    const double den = it == 0 ? delta : delta - beta * gamma / alpha_prev;
    if (!(den > 0.0) || !(gamma > 0.0)) { o.status = EGFEM_BREAKDOWN; break; }
    const double alpha = gamma / den;
    p = fma(beta, p, u);
    sv = fma(beta, sv, wv);
    x = fma(alpha, p, x);
    r = fma(-alpha, sv, r);
    if (!own) r = 0.0;
    if (!exact && rnorm <= kCgExact * ref) exact = true;   // from this update on
    if (!exact) {
      shv = fma(beta, shv, wh);
      u = own ? fma(-alpha, shv, u) : 0.0;
      xu[tid] = u;
      if (gown) {
        const double gw = ll_value(ww.lo, ww.hi);
        gs = fma(beta, gs, gw);
        gu = fma(-alpha, gs, gu);
        xu[NT + 1 + tid] = gu;
      }
    } else {
      // u = M^-1 r, published for the ghosts
      const double xs[1] = {r};
      double zs[1];
      ov_prec<NT, K, 1>(li, ab, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
      u = own ? zs[0] : 0.0;
      ++ep;
      const unsigned fu = ll_flag(O.salt, ep);
      if (own) ll_store(llu + 2 * (size_t)row, u, fu);
      xu[tid] = u;
      GhostWords wu;
      if (ng > 0) ghost_load(llu, gc, wu);
      const bool gab = ng > 0 && ghost_wait(llu, gc, fu, wu, abort_word);
      if ((o.abort = wg_any(gab, &sh_state[1]))) break;
      if (gown) {
        gu = ll_value(wu.lo, wu.hi);
        xu[NT + 1 + tid] = gu;
      }
    }
    gamma_prev = gamma;
    alpha_prev = alpha;
    ++it;
    lds_barrier();
  }
#undef EGFEM_ZERO_RED
  if (!o.abort && own) A.x[row] = x;
  o.iters = it;
  o.rnorm = rnorm;
  o.bnorm = ref;
  return o;
}

}  // namespace dev
}  // namespace egfem
