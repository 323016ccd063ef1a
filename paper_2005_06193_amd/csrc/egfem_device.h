// Device building blocks shared by the single-instance kernels and the
// batched persistent Newton kernel:
//   * row-block tensor stages (residual action, Jacobian emission),
//   * team barrier and deterministic team reductions,
//   * the Jacobi-BiCGStab iteration run by a team of workgroups.
// A "team" is a set of co-resident workgroups that synchronise among
// themselves only (one team = the whole grid for a single solve; one team per
// instance in the batched kernel).
#pragma once

#include <type_traits>

#include "egfem_internal.h"

namespace egfem {
namespace dev {

constexpr int kWave = 64;
constexpr unsigned kSpinCap = 1u << 24;   // bounded waits: a barrier that never completes aborts
constexpr int kGroups = 32;               // most arrival groups of a team barrier
// control block (unsigned words, one 128-byte line each): epoch, global
// arrivals, abort flag, then one arrival counter per group.
constexpr int kCtrlGen = 0, kCtrlAll = 32, kCtrlAbort = 64, kCtrlGroup = 96;
constexpr int kCtrlFlags = kCtrlGroup + 32 * kGroups;   // one publication flag per workgroup
constexpr int kCtrlWords = kCtrlFlags + kMaxKrylovBlocks;
constexpr int kMaxNbr = kMaxNbrLists;     // most neighbours of a point-to-point synchronisation
static_assert(kCtrlWords <= kCtrlWordsMax, "barrier control block too small");
constexpr int kMaxRed = 8;                // values per reduction

// Agent-coherent accessors for data exchanged between workgroups.
__device__ __forceinline__ double ld_sh(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Agent-coherent store at a 32-bit byte offset from a uniform base: the base
// stays in scalar registers and the address is formed by the store itself,
// so no 64-bit per-lane address has to be kept in vector registers.
// (The base is a global-memory pointer: in that address space the access
// takes the scalar-base plus 32-bit-offset addressing of global instructions.)
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ void st_sh_at(double* base, unsigned off, double v) {
  gchar* b = (gchar*)base;
  __asm__ volatile("" : "+s"(b));
  __hip_atomic_store((gdouble*)(b + off), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_sh_at(const double* base, unsigned off) {
  const gchar* b = (const gchar*)base;
  __asm__ volatile("" : "+s"(b));
  return __hip_atomic_load((const gdouble*)(b + off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Plain (row-local) load and store at a 32-bit byte offset from a uniform base.
__device__ __forceinline__ void st_at(double* base, unsigned off, double v) {
  gchar* b = (gchar*)base;
  __asm__ volatile("" : "+s"(b));
  *(gdouble*)(b + off) = v;
}
__device__ __forceinline__ double ld_at(const double* base, unsigned off) {
  const gchar* b = (const gchar*)base;
  __asm__ volatile("" : "+s"(b));
  return *(const gdouble*)(b + off);
}
template <bool SH>
__device__ __forceinline__ double ld(const double* p) {
  return SH ? ld_sh(p) : *p;
}

// ---------------------------------------------------------------------------
// Tensor view and row-block stages
// ---------------------------------------------------------------------------
struct TensorView {
  int64_t n;
  int64_t nblk;
  int sym;
  const int32_t* blk_row;
  const int4* meta;         // two int4 per block: r0 r1 s0 s1 | pa0 pa1 pb0 pb1
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* kptrA;
  const int32_t* kA;
  const double* vA;
  const int32_t* jptrB;
  const int32_t* jB;
  const double* vB;
  const uint16_t* kS;       // block-relative slot of (i, k) of every A entry
  const uint16_t* bS;       // block-relative B position of every A entry (not symmetric)
  const uint16_t* kpS;      // A fiber start relative to the block's first A entry
  const uint16_t* jpS;      // B fiber start relative to the block's first B entry
  const double* kval;
  // W_h = P2 (Case 1): A entries name k by the block-relative W-slot; the B
  // stream is aligned to W-slots (jpS per W-slot)
  const int2* wmeta;        // W-slot range of every block
  const int32_t* wrowptr;   // W-slot range of every row
  const int32_t* wcol;      // P2 dof of every W-slot
  const uint32_t* wpq;      // block-relative slots of a W-slot's endpoints, p | q << 16
  // W_h = I_k (Case 3): a W-slot is a quadrature point of a cell of the row;
  // wpq / wpq2 hold the slots of the cell's vertices, qlam their barycentrics
  const uint32_t* wpq2;     // slots of the third and fourth vertex
  const uint8_t* wqi;       // point index of every W-slot
  const double* qlam;       // [4][4] barycentrics of the points
  // symmetric half stream (T_ijk = T_ikj): k at or after j, diagonal halved
  const uint16_t* kSH;
  const double* vH;
  const uint16_t* kpSH;
  const int2* hmeta;
};

// Bounds of row block b: rows [r0, r1), slots [s0, s1), A entries [pa0, pa1),
// B entries [pb0, pb1).  b is uniform, so this is one scalar load.
struct BlockMeta {
  int r0, r1, s0, s1, pa0, pa1, pb0, pb1;
};
__device__ __forceinline__ BlockMeta block_meta(const TensorView& T, int64_t b) {
  const int4 x = T.meta[2 * b], y = T.meta[2 * b + 1];
  return BlockMeta{x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
}

// LDS scratch of the row-block stages (one block at a time per workgroup).
struct RowBlockLds {
  double tA[kCapNnz];        // products of the A stream
  double tB[kCapNnz];        // products of the B stream (Jacobian only)
  double aS[kCapSlots];      // a at every slot's column
  double uS[kCapSlots];      // u at every slot's column (Jacobian only)
  double y[kCapSlots];       // slot results (action)
  int spa[kCapSlots + 1];    // fiber bounds, A stream, block-relative
  int spb[kCapSlots + 1];    // fiber bounds, B stream, block-relative
  int srow[kCapRows + 1];    // slot bounds of the rows, block-relative
  int srid[kCapSlots];       // row of every slot, block-relative (Jacobian)
  uint16_t pslot[kCapNnz];   // slot of every A entry, block-relative (Jacobian)
  unsigned char sdir[kCapRows];
};

// LDS scratch of the Jacobian emission alone (no action stages, 16-bit
// bounds and indices; at most kCapNnz entries and kCapSlots slots per block):
// 29 KiB, five 256-thread workgroups per CU where RowBlockLds allows four.
struct JacobianLds {
  double tA[kCapNnz];
  double tB[kCapNnz];
  double aS[kCapSlots];
  double uS[kCapSlots];
  uint16_t spa[kCapSlots + 1];
  uint16_t spb[kCapSlots + 1];
  uint16_t srid[kCapSlots];
  uint16_t pslot[kCapNnz];
  unsigned char sdir[kCapRows];
};

// LDS scratch of the residual action alone (smaller: higher occupancy).
struct ActionLds {
  double tA[kCapNnz];
  double aS[kCapSlots];
  double y[kCapSlots];
  int spa[kCapSlots + 1];
  int srow[kCapRows + 1];
};

// Entries / slots one thread handles in a row block.
template <int NT>
struct Per {
  static_assert(NT >= kCapRows, "one thread per row of a block");
  static constexpr int P = (kCapNnz + NT - 1) / NT;
  static constexpr int S = (kCapSlots + NT - 1) / NT;
};

// Stream registers of one row block for the tensor action (stage 1a).
template <int NT>
struct ActionRegs {
  int kk[Per<NT>::P];       // block-relative slot of (i, k)
  double vv[Per<NT>::P];
  int cc[Per<NT>::S];
  int kp[Per<NT>::S];       // fiber start relative to the block's first entry
  double kv[Per<NT>::S];
  int r0, s0, p0, np, ns, nr, rp;
  double ldi;
  unsigned char dr;
};

// Loads are issued without per-entry branches: a load under a divergent
// branch is followed by a wait for its value (the branch merge copies it), so
// a thread's loads would complete one after the other.  Indices past the end
// of a range are clamped to its last element (the streams are padded, so even
// an empty range clamps in bounds) and the extra values are masked at use.
__device__ __forceinline__ int clamp_hi(int x, int n) { return min(x, max(n - 1, 0)); }

// acc + x[lo] + x[lo+1] + ... + x[hi-1], added in that order (the result of
// the plain loop, bit for bit), with the LDS reads issued four at a time:
// reads past hi are clamped to hi - 1 and their values not added, so four
// reads are in flight per wait instead of one.
__device__ __forceinline__ double lds_range_sum(const double* x, int lo, int hi, double acc) {
  for (int t = lo; t < hi; t += 4) {
    const double v0 = x[t];
    const double v1 = x[min(t + 1, hi - 1)];
    const double v2 = x[min(t + 2, hi - 1)];
    const double v3 = x[min(t + 3, hi - 1)];
    acc += v0;
    if (t + 1 < hi) acc += v1;
    if (t + 2 < hi) acc += v2;
    if (t + 3 < hi) acc += v3;
  }
  return acc;
}

// Stage 1a of the tensor action: every stream load of this thread for block b
// (its entries, slots and row), issued back to back without waiting.
template <int NT, bool PROBLEM>
__device__ __forceinline__ void action_load(const TensorView& T, int64_t b, const double* load,
                                            const uint8_t* dir, const double* kval, ActionRegs<NT>& R) {
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S;
  const int tid = threadIdx.x;
  const BlockMeta m = block_meta(T, b);
  R.r0 = m.r0;
  R.s0 = m.s0;
  R.p0 = m.pa0;
  R.np = m.pa1 - m.pa0;
  R.ns = m.s1 - m.s0;
  R.nr = m.r1 - m.r0;
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = R.p0 + clamp_hi(tid + q * NT, R.np);
    R.kk[q] = T.kS[p];
    R.vv[q] = T.vA[p];
  }
  // null kval / load / dir are replaced by a valid array and masked at use;
  // their loads then all read its first word (one cache line, no stream traffic)
  const double* kvp = kval ? kval : T.kval;
  const int kmask = kval ? -1 : 0;   // no K: every lane reads one word (masked at use)
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = R.s0 + clamp_hi(tid + q * NT, R.ns);
    R.cc[q] = T.col[s];
    R.kp[q] = T.kpS[s];
    R.kv[q] = PROBLEM ? kvp[s & kmask] : 0.0;
  }
  const int i = R.r0 + clamp_hi(tid, R.nr);
  R.rp = T.rowptr[i];
  R.ldi = 0.0;
  R.dr = 0;
  if (PROBLEM) {
    R.ldi = (load ? load : T.kval)[load ? i : 0];
    R.dr = (dir ? dir : reinterpret_cast<const uint8_t*>(T.kval))[dir ? i : 0];
  }
}

// Stages 1b-3 of the tensor action on the registers of one block:
//   r_i = sum_{s in row i} w_col(s) * (sum_{p in A(s)} v_p a_{k_p} [+ K_s])
//   RAW:     a given;                                     out = r
//   PROBLEM: a = a0 + w^2, w = u + alpha delta (delta may be null);
//            out = F = r - load, Dirichlet rows 0; uout (optional) = w;
//            sq += F_i^2 over the rows this thread handled.
// SH: u, delta gathered with agent-coherent loads, out and uout written with
// agent-coherent stores (data produced or read by other workgroups of the same
// launch).
// Gathers are per slot (w and a at the slot's column, a into LDS); an entry
// reads a_k from the LDS slot of (i, k).
template <int NT, bool PROBLEM, bool SH, typename Lds>
__device__ __forceinline__ void action_compute(const ActionRegs<NT>& R, const double* u,
                                               const double* delta, double alpha, const double* a,
                                               double a0c, const double* kval, const double* load,
                                               const uint8_t* dir, double* out, double* uout, double& sq,
                                               Lds& L) {
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S;
  const int tid = threadIdx.x;
  const bool has_row = tid < R.nr;
  const int i = R.r0 + clamp_hi(tid, R.nr);
  // per-slot gathers
  double wj[SS], dj[SS], aj[SS];
  double ui = 0.0, di = 0.0;
#pragma unroll
  for (int q = 0; q < SS; ++q) wj[q] = ld<SH>(u + R.cc[q]);
  if (a) {
#pragma unroll
    for (int q = 0; q < SS; ++q) aj[q] = a[R.cc[q]];
  }
  if (PROBLEM && uout) ui = ld<SH>(u + i);
  if (PROBLEM && delta) {
#pragma unroll
    for (int q = 0; q < SS; ++q) dj[q] = ld<SH>(delta + R.cc[q]);
    if (uout) di = ld<SH>(delta + i);
  }
  // slot values (a in LDS) and bounds
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    double as;
    if (PROBLEM) {
      if (delta) wj[q] = fma(alpha, dj[q], wj[q]);
      as = fma(wj[q], wj[q], a ? aj[q] : a0c);
    } else {
      as = aj[q];
    }
    if (s < R.ns) {
      L.aS[s] = as;
      L.spa[s] = R.kp[q];
    }
  }
  if (tid == 0) {
    L.spa[R.ns] = R.np;
    L.srow[R.nr] = R.ns;
  }
  if (has_row) L.srow[tid] = R.rp - R.s0;
  __syncthreads();
  // products
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = tid + q * NT;
    if (p < R.np) L.tA[p] = R.vv[q] * L.aS[R.kk[q]];
  }
  __syncthreads();
  // fiber sums (same slots as loaded by this thread)
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < R.ns) {
      double acc = lds_range_sum(L.tA, L.spa[s], L.spa[s + 1], 0.0);
      if (PROBLEM && kval) acc += R.kv[q];
      L.y[s] = acc * wj[q];
    }
  }
  __syncthreads();
  // row sums
  if (has_row) {
    double acc = lds_range_sum(L.y, L.srow[tid], L.srow[tid + 1], 0.0);
    if (PROBLEM) {
      const bool drow = dir && R.dr;
      if (load) acc -= R.ldi;
      if (drow) acc = 0.0;
      if (uout) {
        double wi = delta ? fma(alpha, di, ui) : ui;
        wi = drow ? 0.0 : wi;
        if (SH) st_sh(uout + i, wi);
        else uout[i] = wi;
      }
      sq = fma(acc, acc, sq);
    }
    if (SH) st_sh(out + i, acc);   // read by other workgroups of the launch (batched)
    else out[i] = acc;
  }
  __syncthreads();   // LDS is reused by the next block
}

// Tensor action over row block b with NT threads (load + compute).
template <int NT, bool PROBLEM, bool SH, typename Lds>
__device__ void rowblock_action(const TensorView& T, int64_t b, const double* u, const double* delta,
                                double alpha, const double* a, double a0c, const double* load,
                                const uint8_t* dir, const double* kval, double* out, double* uout,
                                double& sq, Lds& L) {
  ActionRegs<NT> R;
  action_load<NT, PROBLEM>(T, b, load, dir, kval, R);
  action_compute<NT, PROBLEM, SH>(R, u, delta, alpha, a, a0c, kval, load, dir, out, uout, sq, L);
}

// Tensor action over the contiguous block range [b0, b1) of one workgroup,
// one block after the other (no prefetch: fewer registers, higher occupancy).
template <int NT, bool PROBLEM, bool SH, typename Lds>
__device__ void rowblocks_action(const TensorView& T, int64_t b0, int64_t b1, const double* u,
                                 const double* delta, double alpha, const double* a, double a0c,
                                 const double* load, const uint8_t* dir, const double* kval, double* out,
                                 double* uout, double& sq, Lds& L) {
  for (int64_t b = b0; b < b1; ++b)
    rowblock_action<NT, PROBLEM, SH>(T, b, u, delta, alpha, a, a0c, load, dir, kval, out, uout, sq, L);
}

// Tensor action over the contiguous block range [b0, b1) of one workgroup,
// software-pipelined: the stream loads of block b+1 are issued before the
// gathers and LDS stages of block b, so they overlap that dependent chain.
template <int NT, bool PROBLEM, bool SH, typename Lds>
__device__ void rowblocks_action_pipelined(const TensorView& T, int64_t b0, int64_t b1, const double* u,
                                           const double* delta, double alpha, const double* a,
                                           double a0c, const double* load, const uint8_t* dir,
                                           const double* kval, double* out, double* uout, double& sq,
                                           Lds& L) {
  if (b0 >= b1) return;
  // two named register sets (a dynamically indexed pair would live in scratch)
  ActionRegs<NT> RA, RB;
  action_load<NT, PROBLEM>(T, b0, load, dir, kval, RA);
  for (int64_t b = b0; b < b1; b += 2) {
    if (b + 1 < b1) action_load<NT, PROBLEM>(T, b + 1, load, dir, kval, RB);
    action_compute<NT, PROBLEM, SH>(RA, u, delta, alpha, a, a0c, kval, load, dir, out, uout, sq, L);
    if (b + 1 >= b1) break;
    if (b + 2 < b1) action_load<NT, PROBLEM>(T, b + 2, load, dir, kval, RA);
    action_compute<NT, PROBLEM, SH>(RB, u, delta, alpha, a, a0c, kval, load, dir, out, uout, sq, L);
  }
}

// Jacobian emission over row block b with NT threads:
//   J_s = [K_s] + sum_{p in A(s)} v_p a_{k_p} + g_j sum_{p in B(s)} v_p u_{j_p},
// s = (i, j), a = a0 + u^2 (problem_a) or given, g = dadu or 2u (dadu_2u) or none.
// Dirichlet rows -> identity rows, Dirichlet columns -> 0; dinv[i] = 1 / J_ii.
// Two phases: every thread loads its A entries, slots and row, gathers and
// writes products and bounds to LDS; then every slot sums its two fibers and
// stores J_s (coalesced).  The B fiber of slot (i, k) holds the A entries
// (i, j, k) of the row; each A entry places its second product v u_j (u at
// the column of the slot that holds it) at its B position, so the B stream
// is read as one 16-bit position per entry and the sums run in B order.
template <int NT, bool SH, typename Lds>
__device__ void rowblock_jacobian(const TensorView& T, int64_t b, const double* u, const double* a,
                                  const double* a0, double a0c, int problem_a, const double* dadu,
                                  int dadu_2u, const double* kval, const uint8_t* dir, double* jval,
                                  double* dinv, Lds& L) {
  static_assert(NT >= kCapRows, "one thread per row of a block");
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S;
  const int tid = threadIdx.x;
  const BlockMeta m = block_meta(T, b);
  const int r0 = m.r0, s0 = m.s0, pa0 = m.pa0;
  const int na = m.pa1 - m.pa0, nb = m.pb1 - m.pb0, ns = m.s1 - m.s0, nr = m.r1 - m.r0;
  const bool second = dadu || dadu_2u;
  const bool bstream = second && !T.sym;
  const bool need_u = problem_a || second;
  // stage 1a: stream loads, back to back at clamped indices (see action_load);
  // entries name their k by the block-relative slot of (i, k) and, without the
  // symmetry, their place in the B stream by a block-relative position
  int ka[PP], bp[PP];
  double va[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = pa0 + clamp_hi(tid + q * NT, na);
    ka[q] = T.kS[p];
    va[q] = T.vA[p];
    if (bstream) bp[q] = T.bS[p];
  }
  int cc[SS], kpa[SS], kpe[SS], kpb[SS];
  double kv[SS];
  const double* kvp = kval ? kval : T.kval;
  const int kmask = kval ? -1 : 0;   // no K: every lane reads one word (masked at use)
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int sl = tid + q * NT;
    const int s = s0 + clamp_hi(sl, ns);
    cc[q] = T.col[s];
    kpa[q] = T.kpS[s];
    kpb[q] = T.jpS[s];   // symmetric: aliases kpS
    // end of the slot's A fiber (kpS has one entry past the last slot)
    kpe[q] = bstream ? (sl + 1 < ns ? (int)T.kpS[s + 1] : na) : 0;
    kv[q] = kvp[s & kmask];
  }
  const bool has_row = tid < nr;
  const int i = r0 + clamp_hi(tid, nr);
  const int rpa = T.rowptr[i], rpb = T.rowptr[i + 1];
  const unsigned char drow_raw = (dir ? dir : reinterpret_cast<const uint8_t*>(T.kval))[dir ? i : 0];
  // stage 1b: per-slot gathers (u, a or a0, g, Dirichlet flag at the slot's column)
  double uj[SS], aj[SS], gj[SS];
  unsigned char dcr[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    uj[q] = 0.0;
    gj[q] = 0.0;
    dcr[q] = 0;
  }
  if (need_u) {
#pragma unroll
    for (int q = 0; q < SS; ++q) uj[q] = ld<SH>(u + cc[q]);
  }
  const double* ga = problem_a ? a0 : a;   // a0 may be null (constant a0c)
  if (ga) {
#pragma unroll
    for (int q = 0; q < SS; ++q) aj[q] = ga[cc[q]];
  }
  if (dadu) {
#pragma unroll
    for (int q = 0; q < SS; ++q) gj[q] = dadu[cc[q]];
  }
  if (dir) {
#pragma unroll
    for (int q = 0; q < SS; ++q) dcr[q] = dir[cc[q]];
  }
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      L.aS[s] = problem_a ? fma(uj[q], uj[q], a0 ? aj[q] : a0c) : aj[q];
      L.uS[s] = uj[q];
      L.spa[s] = kpa[q];
      L.spb[s] = kpb[q];
      if (bstream)
        for (int p = kpa[q]; p < kpe[q]; ++p) L.pslot[p] = (uint16_t)s;
    }
  }
  if (tid == 0) {
    L.spa[ns] = na;
    L.spb[ns] = nb;
  }
  if (has_row) {
    L.sdir[tid] = (dir && drow_raw) ? 1 : 0;
    for (int s = rpa - s0; s < rpb - s0; ++s) L.srid[s] = tid;
  }
  __syncthreads();
  // stage 1c: products
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = tid + q * NT;
    if (p < na) {
      L.tA[p] = va[q] * L.aS[ka[q]];
      if (T.sym && second) L.tB[p] = va[q] * L.uS[ka[q]];
      if (bstream) L.tB[bp[q]] = va[q] * L.uS[L.pslot[p]];
    }
  }
  __syncthreads();
  // stage 2: slot assembly
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      const int ir = L.srid[s];
      const int row = r0 + ir;
      const int j = cc[q];
      double J;
      if (L.sdir[ir]) {
        J = (j == row) ? 1.0 : 0.0;
      } else if (dcr[q]) {
        J = 0.0;
      } else {
        const double qa = lds_range_sum(L.tA, L.spa[s], L.spa[s + 1], 0.0);
        J = (kval ? kv[q] : 0.0) + qa;
        if (second) {
          const double qb = lds_range_sum(L.tB, L.spb[s], L.spb[s + 1], 0.0);
          const double g = dadu ? gj[q] : 2.0 * uj[q];
          J = fma(g, qb, J);
        }
      }
      // SH: other workgroups of the launch may read these rows (batched)
      if (SH) st_sh(jval + s0 + s, J);
      else jval[s0 + s] = J;
      if (j == row && dinv) {
        if (SH) st_sh(dinv + row, 1.0 / J);
        else dinv[row] = 1.0 / J;
      }
    }
  }
  __syncthreads();   // LDS is reused by the next block
}

// ---------------------------------------------------------------------------
// Tensor action from the symmetric half stream (T_ijk = T_ikj)
// ---------------------------------------------------------------------------
// With h_ijk = T_ijk for k after j and T_ijj / 2 on the diagonal,
//   r_i = sum_j sum_k T_ijk w_j a_k = sum_j [ w_j sum_{k>=j} h_ijk a_k + a_j sum_{k>=j} h_ijk w_k ],
// so each slot sums two products of its half fiber.
struct ActionLdsH {
  double tA[kCapNnz];
  double tU[kCapNnz];
  double aS[kCapSlots];
  double wS[kCapSlots];
  double y[kCapSlots];
  int spa[kCapSlots + 1];
  int srow[kCapRows + 1];
};

template <int NT, bool PROBLEM>
__device__ void rowblock_action_half(const TensorView& T, int64_t b, const double* u, const double* delta,
                                     double alpha, const double* a, double a0c, const double* load,
                                     const uint8_t* dir, const double* kval, double* out, double* uout,
                                     double& sq, ActionLdsH& L) {
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S;
  const int tid = threadIdx.x;
  const BlockMeta m = block_meta(T, b);
  const int2 hm = T.hmeta[b];
  const int np = hm.y - hm.x, ns = m.s1 - m.s0, nr = m.r1 - m.r0;
  int kk[PP];
  double vv[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = hm.x + clamp_hi(tid + q * NT, np);
    kk[q] = T.kSH[p];
    vv[q] = T.vH[p];
  }
  const double* kvp = kval ? kval : T.kval;
  const int kmask = kval ? -1 : 0;   // no K: every lane reads one word (masked at use)
  int cc[SS], kp[SS];
  double kv[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = m.s0 + clamp_hi(tid + q * NT, ns);
    cc[q] = T.col[s];
    kp[q] = T.kpSH[s];
    kv[q] = kvp[s & kmask];
  }
  const bool has_row = tid < nr;
  const int i = m.r0 + clamp_hi(tid, nr);
  const int rp = T.rowptr[i];
  const double ldi = (PROBLEM && load) ? load[i] : 0.0;
  const unsigned char dr = (PROBLEM && dir) ? dir[i] : 0;
  double wj[SS], aj[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    wj[q] = u[cc[q]];
    if (PROBLEM && delta) wj[q] = fma(alpha, delta[cc[q]], wj[q]);
    aj[q] = PROBLEM ? fma(wj[q], wj[q], a ? a[cc[q]] : a0c) : a[cc[q]];
  }
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      L.wS[s] = wj[q];
      L.aS[s] = aj[q];
      L.spa[s] = kp[q];
    }
  }
  if (tid == 0) {
    L.spa[ns] = np;
    L.srow[nr] = ns;
  }
  if (has_row) L.srow[tid] = rp - m.s0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = tid + q * NT;
    if (p < np) {
      L.tA[p] = vv[q] * L.aS[kk[q]];
      L.tU[p] = vv[q] * L.wS[kk[q]];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      double sa = 0.0, su = 0.0;
      for (int t = L.spa[s]; t < L.spa[s + 1]; ++t) {
        sa += L.tA[t];
        su += L.tU[t];
      }
      if (PROBLEM && kval) sa += kv[q];
      L.y[s] = fma(aj[q], su, sa * wj[q]);
    }
  }
  __syncthreads();
  if (has_row) {
    double acc = 0.0;
    for (int t = L.srow[tid]; t < L.srow[tid + 1]; ++t) acc += L.y[t];
    if (PROBLEM) {
      const bool drow = dir && dr;
      if (load) acc -= ldi;
      if (drow) acc = 0.0;
      if (uout) {
        const double wi = delta ? fma(alpha, delta[i], u[i]) : u[i];
        uout[i] = drow ? 0.0 : wi;
      }
      sq = fma(acc, acc, sq);
    }
    out[i] = acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Row-block stages for a coefficient space W_h != V_h: WK = 1 P2 (Case 1 of
// Sec. 3.1), WK = 2 the quadrature-point space I_k (Case 3)
// ---------------------------------------------------------------------------
// The coefficient lives on the P2 dofs.  Every P2 dof k coupled to row i is a
// vertex or an edge of a cell of i, so both of its endpoints are columns of
// row i: the interpolation Pi_u of Sec. 3.2 (vertex value, or the mean of the
// two endpoint values) is formed from the per-slot gathers, and
// a_k = (Pi a0)_k + ((Pi w)_k)^2 is computed once per W-slot in LDS.
constexpr int kPerW(int nt) { return (kCapWSlots + nt - 1) / nt; }

struct ActionLdsW {
  double tA[kCapNnz];
  double aS[kCapWSlots];     // a at every W-slot
  double wS[kCapSlots];      // w at every slot's column
  double zS[kCapSlots];      // a0 at every slot's column
  double y[kCapSlots];
  int spa[kCapSlots + 1];
  int srow[kCapRows + 1];
};

__device__ __forceinline__ int w_lo(uint32_t pq) { return (int)(pq & 0xffffu); }
__device__ __forceinline__ int w_hi(uint32_t pq) { return (int)(pq >> 16); }

// Tensor action of row block b (one block per workgroup):
//   RAW:     r_i = sum_{s=(i,j)} w_j sum_{p in A(s)} v_p a_{k_p}, a given on the P2 dofs;
//   PROBLEM: a = Pi a0 + (Pi w)^2 with w = u + alpha delta, a0 nodal (or a0c);
//            F = r [+ K w] - load, Dirichlet rows 0, uout = w, sq += F_i^2.
template <int NT, bool PROBLEM, int WK>
__device__ void rowblock_action_w2(const TensorView& T, int64_t b, const double* u, const double* delta,
                                   double alpha, const double* a, double a0c, const double* load,
                                   const uint8_t* dir, const double* kval, double* out, double* uout,
                                   double& sq, ActionLdsW& L) {
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S, WW = kPerW(NT);
  const int tid = threadIdx.x;
  const BlockMeta m = block_meta(T, b);
  const int2 wm = T.wmeta[b];
  const int np = m.pa1 - m.pa0, ns = m.s1 - m.s0, nr = m.r1 - m.r0, nw = wm.y - wm.x;
  // stream loads at clamped indices
  int kk[PP];
  double vv[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = m.pa0 + clamp_hi(tid + q * NT, np);
    kk[q] = T.kS[p];
    vv[q] = T.vA[p];
  }
  const double* kvp = kval ? kval : T.kval;
  const int kmask = kval ? -1 : 0;   // no K: every lane reads one word (masked at use)
  int cc[SS], kp[SS];
  double kv[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = m.s0 + clamp_hi(tid + q * NT, ns);
    cc[q] = T.col[s];
    kp[q] = T.kpS[s];
    kv[q] = kvp[s & kmask];
  }
  uint32_t wq[WW], wq2[WW];
  int wc[WW], wqq[WW];
#pragma unroll
  for (int q = 0; q < WW; ++q) {
    const int w = wm.x + clamp_hi(tid + q * NT, nw);
    if (PROBLEM) {
      wq[q] = T.wpq[w];
      if (WK == 2) {
        wq2[q] = T.wpq2[w];
        wqq[q] = T.wqi[w];
      }
    } else {
      wc[q] = T.wcol[w];
    }
  }
  const bool has_row = tid < nr;
  const int i = m.r0 + clamp_hi(tid, nr);
  const int rp = T.rowptr[i];
  const double ldi = (PROBLEM && load) ? load[i] : 0.0;
  const unsigned char dr = (PROBLEM && dir) ? dir[i] : 0;
  // per-slot gathers
  double wj[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    wj[q] = u[cc[q]];
    if (PROBLEM && delta) wj[q] = fma(alpha, delta[cc[q]], wj[q]);
  }
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      L.wS[s] = wj[q];
      if (PROBLEM) L.zS[s] = a ? a[cc[q]] : a0c;
      L.spa[s] = kp[q];
    }
  }
  if (!PROBLEM) {
#pragma unroll
    for (int q = 0; q < WW; ++q) {
      const int t = tid + q * NT;
      if (t < nw) L.aS[t] = a[wc[q]];
    }
  }
  if (tid == 0) {
    L.spa[ns] = np;
    L.srow[nr] = ns;
  }
  if (has_row) L.srow[tid] = rp - m.s0;
  __syncthreads();
  if (PROBLEM) {
#pragma unroll
    for (int q = 0; q < WW; ++q) {
      const int t = tid + q * NT;
      if (t < nw) {
        const int p0 = w_lo(wq[q]), p1 = w_hi(wq[q]);
        double pw, pz;
        if (WK == 1) {
          pw = 0.5 * (L.wS[p0] + L.wS[p1]);
          pz = 0.5 * (L.zS[p0] + L.zS[p1]);
        } else {
          const int p2 = w_lo(wq2[q]), p3 = w_hi(wq2[q]);
          const double* lam = T.qlam + 4 * wqq[q];
          pw = fma(lam[3], L.wS[p3], fma(lam[2], L.wS[p2], fma(lam[1], L.wS[p1], lam[0] * L.wS[p0])));
          pz = fma(lam[3], L.zS[p3], fma(lam[2], L.zS[p2], fma(lam[1], L.zS[p1], lam[0] * L.zS[p0])));
        }
        L.aS[t] = fma(pw, pw, pz);
      }
    }
    __syncthreads();
  }
  // products
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = tid + q * NT;
    if (p < np) L.tA[p] = vv[q] * L.aS[kk[q]];
  }
  __syncthreads();
  // fiber sums times w_j
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      double acc = 0.0;
      for (int t = L.spa[s]; t < L.spa[s + 1]; ++t) acc += L.tA[t];
      if (PROBLEM && kval) acc += kv[q];
      L.y[s] = acc * wj[q];
    }
  }
  __syncthreads();
  // row sums
  if (has_row) {
    double acc = 0.0;
    for (int t = L.srow[tid]; t < L.srow[tid + 1]; ++t) acc += L.y[t];
    if (PROBLEM) {
      const bool drow = dir && dr;
      if (load) acc -= ldi;
      if (drow) acc = 0.0;
      if (uout) {
        double wi = delta ? fma(alpha, delta[i], u[i]) : u[i];
        uout[i] = drow ? 0.0 : wi;
      }
      sq = fma(acc, acc, sq);
    }
    out[i] = acc;
  }
  __syncthreads();
}

struct RowBlockLdsW {
  double tA[kCapNnz];
  double tB[kCapNnz];
  double aS[kCapWSlots];     // a at every W-slot
  double cW[kCapWSlots];     // g at every W-slot, then g times its B fiber sum
  double uS[kCapSlots];
  double zS[kCapSlots];      // a0 at every slot's column
  double bacc[kCapSlots];    // second term gathered back to the slots
  uint32_t wpq[kCapWSlots];
  int spa[kCapSlots + 1];
  int spbw[kCapWSlots + 1];  // B fiber bounds of every W-slot
  int srow[kCapRows + 1];
  int swrow[kCapRows + 1];   // W-slot bounds of every row
  int srid[kCapSlots];
  uint16_t pslot[kCapNnz];   // slot of every A entry, block-relative
  unsigned char sdir[kCapRows];
};

// Jacobian emission of row block b for W_h = P2:
//   J_s = [K_s] + sum_{p in A(s)} v_p a_{k_p} + sum_k q_ik g_k (Pi_u)_kj,
//   q_ik = sum_{p in B(i,k)} v_p u_{j_p},  s = (i, j),
// a = Pi a0 + (Pi u)^2 (problem_a) or given on the P2 dofs; g = dadu (given on
// the P2 dofs), 2 Pi u (dadu_2u) or none.  (Pi_u)_kj is 1 for the vertex dof
// k = j and 1/2 for an edge dof k with endpoint j.  Every row adds its
// W-slots' terms to its own slots in ascending W-slot order (deterministic).
// Dirichlet rows -> identity rows, Dirichlet columns -> 0; dinv[i] = 1 / J_ii.
template <int NT, int WK>
__device__ void rowblock_jacobian_w2(const TensorView& T, int64_t b, const double* u, const double* a,
                                     const double* a0, double a0c, int problem_a, const double* dadu,
                                     int dadu_2u, const double* kval, const uint8_t* dir, double* jval,
                                     double* dinv, RowBlockLdsW& L) {
  constexpr int PP = Per<NT>::P, SS = Per<NT>::S, WW = kPerW(NT);
  const int tid = threadIdx.x;
  const BlockMeta m = block_meta(T, b);
  const int2 wm = T.wmeta[b];
  const int r0 = m.r0, s0 = m.s0;
  const int na = m.pa1 - m.pa0, nb = m.pb1 - m.pb0, ns = m.s1 - m.s0, nr = m.r1 - m.r0, nw = wm.y - wm.x;
  const bool second = dadu || dadu_2u;
  const bool need_u = problem_a || second;
  // the B fiber of W-slot (i, w) holds the A entries (i, j, w) of the row:
  // each A entry places its product v u_j at its B position (see rowblock_jacobian)
  int ka[PP], bp[PP];
  double va[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = m.pa0 + clamp_hi(tid + q * NT, na);
    ka[q] = T.kS[p];
    va[q] = T.vA[p];
    if (second) bp[q] = T.bS[p];
  }
  int cc[SS], kpa[SS], kpe[SS];
  double kv[SS];
  const double* kvp = kval ? kval : T.kval;
  const int kmask = kval ? -1 : 0;   // no K: every lane reads one word (masked at use)
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int sl = tid + q * NT;
    const int s = s0 + clamp_hi(sl, ns);
    cc[q] = T.col[s];
    kpa[q] = T.kpS[s];
    // end of the slot's A fiber (kpS has one entry past the last slot)
    kpe[q] = second ? (sl + 1 < ns ? (int)T.kpS[s + 1] : na) : 0;
    kv[q] = kvp[s & kmask];
  }
  uint32_t wq[WW], wq2[WW];
  int wc[WW], wbp[WW], wqq[WW];
#pragma unroll
  for (int q = 0; q < WW; ++q) {
    const int w = wm.x + clamp_hi(tid + q * NT, nw);
    wq[q] = T.wpq[w];
    wc[q] = T.wcol[w];
    wbp[q] = T.jpS[w];
    if (WK >= 2) {
      wq2[q] = T.wpq2[w];
      wqq[q] = T.wqi[w];
    }
  }
  const bool has_row = tid < nr;
  const int i = r0 + clamp_hi(tid, nr);
  const int rpa = T.rowptr[i], rpb = T.rowptr[i + 1];
  const int wra = T.wrowptr[i], wrb = T.wrowptr[i + 1];
  const unsigned char drow_raw = dir ? dir[i] : 0;
  // per-slot gathers
  double uj[SS];
  unsigned char dcr[SS];
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    uj[q] = need_u ? u[cc[q]] : 0.0;
    dcr[q] = dir ? dir[cc[q]] : 0;
  }
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      L.uS[s] = uj[q];
      L.zS[s] = (problem_a && a0) ? a0[cc[q]] : a0c;
      L.spa[s] = kpa[q];
      L.bacc[s] = 0.0;
      if (second)
        for (int p = kpa[q]; p < kpe[q]; ++p) L.pslot[p] = (uint16_t)s;
    }
  }
  // per-W-slot values that need no slot data
#pragma unroll
  for (int q = 0; q < WW; ++q) {
    const int t = tid + q * NT;
    if (t < nw) {
      L.wpq[t] = wq[q];
      L.spbw[t] = wbp[q];
      if (!problem_a) L.aS[t] = a[wc[q]];
      // WK = 3 (cells): dadu holds 4 weights per cell, applied in the scatter
      if (dadu) L.cW[t] = (WK == 3) ? 1.0 : dadu[wc[q]];
    }
  }
  if (tid == 0) {
    L.spa[ns] = na;
    L.spbw[nw] = nb;
  }
  if (has_row) {
    L.sdir[tid] = (dir && drow_raw) ? 1 : 0;
    L.srow[tid] = rpa - s0;
    L.swrow[tid] = wra - wm.x;
    for (int s = rpa - s0; s < rpb - s0; ++s) L.srid[s] = tid;
    if (tid == nr - 1) {
      L.srow[nr] = rpb - s0;
      L.swrow[nr] = wrb - wm.x;
    }
  }
  __syncthreads();
  // W-slot values from the slot gathers: a = Pi a0 + (Pi u)^2, g = 2 Pi u
  if (problem_a || dadu_2u) {
#pragma unroll
    for (int q = 0; q < WW; ++q) {
      const int t = tid + q * NT;
      if (t < nw) {
        const int p0 = w_lo(wq[q]), p1 = w_hi(wq[q]);
        double pu, pz;
        if (WK == 1) {
          pu = 0.5 * (L.uS[p0] + L.uS[p1]);
          pz = 0.5 * (L.zS[p0] + L.zS[p1]);
        } else {
          const int p2 = w_lo(wq2[q]), p3 = w_hi(wq2[q]);
          const double* lam = T.qlam + 4 * wqq[q];
          pu = fma(lam[3], L.uS[p3], fma(lam[2], L.uS[p2], fma(lam[1], L.uS[p1], lam[0] * L.uS[p0])));
          pz = fma(lam[3], L.zS[p3], fma(lam[2], L.zS[p2], fma(lam[1], L.zS[p1], lam[0] * L.zS[p0])));
        }
        if (problem_a) L.aS[t] = fma(pu, pu, pz);
        if (dadu_2u && !dadu) L.cW[t] = 2.0 * pu;
      }
    }
    __syncthreads();
  }
  // products
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = tid + q * NT;
    if (p < na) {
      L.tA[p] = va[q] * L.aS[ka[q]];
      if (second) L.tB[bp[q]] = va[q] * L.uS[L.pslot[p]];
    }
  }
  __syncthreads();
  if (second) {
    // c_t = g_t * sum over the B fiber of W-slot t
#pragma unroll
    for (int q = 0; q < WW; ++q) {
      const int t = tid + q * NT;
      if (t < nw) {
        double qb = 0.0;
        for (int x = L.spbw[t]; x < L.spbw[t + 1]; ++x) qb += L.tB[x];
        L.cW[t] *= qb;
      }
    }
    __syncthreads();
    // back to the row's slots through Pi_u, one thread per row, fixed order
    if (has_row) {
      for (int t = L.swrow[tid]; t < L.swrow[tid + 1]; ++t) {
        const uint32_t pq = L.wpq[t];
        const int p0 = w_lo(pq), p1 = w_hi(pq);
        const double c = L.cW[t];
        if (WK >= 2) {
          // I_k: (Pi_u)_kj = lambda_j(x_q) for the cell's vertices; cells (WK = 3):
          // the weights d a_k / d u_j passed per cell
          const uint32_t pq2 = T.wpq2[wm.x + t];
          const double* lam = (WK == 2) ? T.qlam + 4 * T.wqi[wm.x + t] : dadu + 4 * (int64_t)T.wcol[wm.x + t];
          L.bacc[p0] += lam[0] * c;
          L.bacc[p1] += lam[1] * c;
          L.bacc[w_lo(pq2)] += lam[2] * c;
          L.bacc[w_hi(pq2)] += lam[3] * c;
        } else if (p0 == p1) {
          L.bacc[p0] += c;
        } else {
          L.bacc[p0] += 0.5 * c;
          L.bacc[p1] += 0.5 * c;
        }
      }
    }
    __syncthreads();
  }
  // slot assembly
#pragma unroll
  for (int q = 0; q < SS; ++q) {
    const int s = tid + q * NT;
    if (s < ns) {
      const int ir = L.srid[s];
      const int row = r0 + ir;
      const int j = cc[q];
      double J;
      if (L.sdir[ir]) {
        J = (j == row) ? 1.0 : 0.0;
      } else if (dcr[q]) {
        J = 0.0;
      } else {
        double qa = 0.0;
        for (int t = L.spa[s]; t < L.spa[s + 1]; ++t) qa += L.tA[t];
        J = (kval ? kv[q] : 0.0) + qa;
        if (second) J += L.bacc[s];
      }
      jval[s0 + s] = J;
      if (j == row && dinv) dinv[row] = 1.0 / J;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Team barrier and reductions
// ---------------------------------------------------------------------------
struct Team {
  unsigned rank;      // this workgroup's index within the team
  unsigned size;      // workgroups in the team
  unsigned* ctrl;     // kCtrlWords control words (zero before the launch)
  double* red;        // reduction slots [kRedSlots][kMaxRed][size]; 0-7 Krylov, 8-9 Newton
  unsigned epoch;     // barriers passed so far
  const int* nbr = nullptr;   // [count, ranks...] of the workgroups whose rows this one gathers
  unsigned flag_epoch = 0;    // point-to-point publications so far
};

// Arrival at and wait for team barrier number `epoch`, by one thread of the
// workgroup, after the workgroup's stores are complete.  Epoch counting (no
// counter resets): arrivals are counted per group (teams of 16 or more
// workgroups; smaller teams count on the team counter directly), the last of
// each group arrives at the team counter, the last team arrival publishes the
// new epoch, everyone else polls it.  All accesses are relaxed agent-scope atomics; data
// exchanged between workgroups is written and read with agent-coherent
// accesses, so no cache write-back or invalidation is needed.  Returns
// nonzero when the team aborted (a wait exceeded kSpinCap).
__device__ inline int barrier_arrive_wait(const Team& tm, unsigned epoch) {
  unsigned* ctrl = tm.ctrl;
  const unsigned G = tm.size;
  int ab = (int)__hip_atomic_load(ctrl + kCtrlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ab) return ab;
  bool last;
  if (G < 16) {
    // small team: one counter
    const unsigned prev = __hip_atomic_fetch_add(ctrl + kCtrlAll, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == (epoch + 1) * G - 1);
  } else {
    // groups of about 8 workgroups (fewer arrivals serialised on one counter)
    const unsigned ng = min(G / 8u, (unsigned)kGroups);
    const unsigned grp = tm.rank % ng;
    const unsigned gsz = (G - grp + ng - 1) / ng;   // ranks r < G with r % ng == grp
    const unsigned prev = __hip_atomic_fetch_add(ctrl + kCtrlGroup + 32 * grp, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    last = false;
    if (prev == (epoch + 1) * gsz - 1) {
      const unsigned prev2 = __hip_atomic_fetch_add(ctrl + kCtrlAll, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      last = (prev2 == (epoch + 1) * ng - 1);
    }
  }
  if (last) {
    __hip_atomic_store(ctrl + kCtrlGen, epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  unsigned spins = 0;
  while (__hip_atomic_load(ctrl + kCtrlGen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins >= kSpinCap) {
      __hip_atomic_store(ctrl + kCtrlAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 1;
    }
    if ((spins & 1023u) == 0 &&
        __hip_atomic_load(ctrl + kCtrlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return 1;
  }
  return 0;
}

// Team barrier.  Every wave first waits until its own stores are complete
// (s_waitcnt vmcnt(0)).  Returns true when the team aborted.
__device__ inline bool team_barrier(Team& tm, int* sh_abort) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are complete
  __syncthreads();
  const unsigned epoch = tm.epoch++;
  if (threadIdx.x == 0) *sh_abort = barrier_arrive_wait(tm, epoch);
  __syncthreads();
  return *sh_abort != 0;
}

// Point-to-point publication for a gather of rows owned by a few other
// workgroups: every wave's stores are complete, the workgroup's flag
// announces publication number `flag_epoch`, then the workgroup waits for the
// same number on the flags of its neighbours (the workgroups owning columns of
// its rows).  Only the read-after-write order of that gather is enforced; the
// caller keeps a team-wide synchronisation between any read of the published
// vector and its next overwrite.  Without a neighbour list (more than kMaxNbr
// neighbours) this is the team barrier.  Returns true when the team aborted.
__device__ inline bool team_neighbor_sync(Team& tm, int* sh_abort) {
  if (!tm.nbr || tm.nbr[0] < 0) return team_barrier(tm, sh_abort);
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are complete
  __syncthreads();
  const unsigned target = ++tm.flag_epoch;
  unsigned* flags = tm.ctrl + kCtrlFlags;
  if (threadIdx.x < (unsigned)kWave) {
    const int lane = threadIdx.x;
    if (lane == 0) __hip_atomic_store(flags + tm.rank, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ab = 0;
    if (lane < tm.nbr[0]) {
      const unsigned* f = flags + tm.nbr[1 + lane];
      unsigned spins = 0;
      while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins >= kSpinCap) {
          __hip_atomic_store(tm.ctrl + kCtrlAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ab = 1;
          break;
        }
        if ((spins & 1023u) == 0 &&
            __hip_atomic_load(tm.ctrl + kCtrlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ab = 1;
          break;
        }
      }
    }
    ab = __any(ab) ? 1 : 0;
    if (lane == 0) *sh_abort = ab;
  }
  __syncthreads();
  return *sh_abort != 0;
}

// Sum of x over the 64 lanes of a wave, returned in every lane, by DPP lane
// moves (a few cycles per step, unlike an LDS permute): pairs and quads
// (quad_perm), half rows and rows (mirrors), then rows 0+1 and 2+3
// (row_bcast:15) and the two halves (row_bcast:31) leave the total in lane 63,
// which is read back as a scalar.  The order of the additions is fixed.
// Requires all 64 lanes active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_move<0xB1, 0xf>(x);    // quad_perm [1,0,3,2]
  x += dpp_move<0x4E, 0xf>(x);    // quad_perm [2,3,0,1]
  x += dpp_move<0x141, 0xf>(x);   // row_half_mirror
  x += dpp_move<0x140, 0xf>(x);   // row_mirror
  x += dpp_move<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// A value every lane of the wave holds (a reduction total read from LDS),
// moved to scalar registers: the compiler cannot prove it uniform by itself,
// and kept in vector registers it costs one register per lane.
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int NT>
constexpr int kShWords = kMaxRed * (NT / kWave) + kMaxRed;

// Team all-reduce of m <= kMaxRed values (every thread contributes v[q],
// every thread receives the team totals), with one team barrier:
//   1. every wave sums its lanes (wave_sum) into LDS; the waves' stores are
//      complete before the workgroup sync;
//   2. wave 0 adds the wave sums (fixed order), publishes the workgroup's
//      partials in reduction slot `slot` ([q][rank]), arrives and waits;
//   3. wave q (q < m; waves take several values when there are fewer waves
//      than values) reads the G partials of value q at once, adds them in a
//      fixed order (lane l: ranks l, l+64, ...; then wave_sum) and puts the
//      total in LDS for every thread.
// The order of every addition is fixed, so results are reproducible.
template <int NT>
__device__ bool team_reduce(Team& tm, int slot, double (&v)[kMaxRed], int m, double* sh,
                            int* sh_abort) {
  constexpr int NW = NT / kWave;
  const unsigned G = tm.size;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < kMaxRed; ++q) {
    if (q < m) {
      const double x = wave_sum(v[q]);
      if (lane == 0) sh[q * NW + wave] = x;
    }
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are complete
  __syncthreads();
  const unsigned epoch = tm.epoch++;
  // partials at 32-bit byte offsets from a base in scalar registers (the slot
  // and the wave's value index are uniform: read-first-lane says so)
  double* part = tm.red + (size_t)__builtin_amdgcn_readfirstlane(slot) * kMaxRed * G;
  if (wave == 0) {
    if (lane < m) {
      double acc = 0.0;
      for (int w = 0; w < NW; ++w) acc += sh[lane * NW + w];
      st_sh_at(part, ((unsigned)lane * G + tm.rank) * 8u, acc);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (lane == 0) *sh_abort = barrier_arrive_wait(tm, epoch);
  }
  __syncthreads();
  if (*sh_abort) return true;
  const int R = (int)((G + kWave - 1) / kWave);
  for (int q = __builtin_amdgcn_readfirstlane(wave); q < m; q += NW) {
    const double* src = part + (size_t)q * G;
    double acc = 0.0;
    for (int r0 = 0; r0 < R; r0 += 4) {
      double y[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) y[r] = ld_sh_at(src, min((unsigned)(lane + kWave * (r0 + r)), G - 1) * 8u);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if ((unsigned)(lane + kWave * (r0 + r)) < G) acc += y[r];
    }
    acc = wave_sum(acc);
    if (lane == 0) sh[kMaxRed * NW + q] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kMaxRed; ++q)
    if (q < m) v[q] = uniform(sh[kMaxRed * NW + q]);
  __syncthreads();   // sh is reused by the next reduction
  return false;
}

// ---------------------------------------------------------------------------
// Jacobi-BiCGStab run by a team
// ---------------------------------------------------------------------------
struct KArgs {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int32_t* perm;      // non-null: use val[perm[s]] (transposed operator)
  const double* dinv;
  const double* rhs;        // b = rhs_scale * rhs (own rows)
  double rhs_scale;
  double* x;                // written with agent-coherent stores
  int x_zero;
  double *r, *rhat, *p, *v, *s, *t, *z;     // row-local
  double *phat, *rh, *vh;                   // gathered by other workgroups (agent-coherent)
  double rtol;
  int max_iter;
  int rel_r0;               // conjugate gradients: tolerance relative to ||r0|| instead of ||b||
  // block-Jacobi preconditioner (register-resident BiCGStab on a compact partition)
  const int32_t* rlist = nullptr;   // non-null: the workgroup's rows are rlist[rb, re)
  const int16_t* kloc = nullptr;    // [slots] position of the column in the row's part, or -1
  int cheb_steps = 0;               // 0: Jacobi D^-1; k >= 2: k Chebyshev steps on the workgroup's block
  double cheb_ratio = 30.0;         // the steps' interval [lmax / cheb_ratio, lmax]
  // ghosts of every part (the products of the LDS-exchange form; part = workgroup)
  const int16_t* kext = nullptr;    // [slots] part-local position of the column (>= 0) or -1 - ghost index
  const int32_t* gptr = nullptr;    // [G + 1] ghost range of every part (at most NT ghosts)
  const int32_t* gcol = nullptr;    // [ghosts] global column of every ghost
};

struct KOut {
  int status;
  int iters;
  double rnorm;
  double bnorm;
  bool abort;
};

// Rows [rb, re), L lanes per row: f(i, (J x1)_i, (J x2)_i) on lane 0 of each
// row's group (x2 may be null); x1 / x2 gathered coherently when SH.
// A lane's first K entries (slots beg + lane + kL, k < K) are loaded
// unconditionally at clamped slots (every row holds its diagonal, so the clamp
// stays in the row) and masked after: the index, value and gather loads of all
// of them are in flight together.  Entries past K*L finish in a loop (none when
// K*L covers the longest row, as the host's choice of L and K ensures for
// meshes of moderate degree).  L = 1 runs one thread per row: a quarter of the
// passes of L = 4 for the same workgroup.  pre(i) loads the row values f needs
// (issued with the row pointers, so they arrive during the product) and f
// receives them: f(i, (J x1)_i, (J x2)_i, pre(i)).
template <int NT, int L, int K, bool SH, typename Pre, typename Fn>
__device__ __forceinline__ void spmv_rows(const KArgs& A, int rb, int re, const double* __restrict__ x1,
                                          const double* __restrict__ x2, Pre pre, Fn f) {
  constexpr int RPP = NT / L;
  const int sub = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  for (int base = rb; base < re; base += RPP) {
    const int i = base + sub;
    const bool row = i < re;
    const int ic = min(i, re - 1);
    const int beg = A.rowptr[ic], end = A.rowptr[ic + 1];
    const auto pv = pre(ic);
    int c[K], v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = min(beg + lane + k * L, end - 1);
      c[k] = A.col[v[k]];
    }
    if (A.perm) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = A.perm[v[k]];
    }
    double a[K], y[K], z[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = A.val[v[k]];
#pragma unroll
    for (int k = 0; k < K; ++k) y[k] = ld<SH>(x1 + c[k]);
    if (x2) {
#pragma unroll
      for (int k = 0; k < K; ++k) z[k] = ld<SH>(x2 + c[k]);
    }
    double acc1 = 0.0, acc2 = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (row && beg + lane + k * L < end) {
        acc1 = fma(a[k], y[k], acc1);
        if (x2) acc2 = fma(a[k], z[k], acc2);
      }
    }
    if (row) {
      for (int s = beg + lane + K * L; s < end; s += L) {
        const double w = A.perm ? A.val[A.perm[s]] : A.val[s];
        const int cs = A.col[s];
        acc1 = fma(w, ld<SH>(x1 + cs), acc1);
        if (x2) acc2 = fma(w, ld<SH>(x2 + cs), acc2);
      }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
      acc1 += __shfl_xor(acc1, off, L);
      acc2 += __shfl_xor(acc2, off, L);
    }
    if (row && lane == 0) f(i, acc1, acc2, pv);
  }
}

// Preconditioned BiCGStab (van der Vorst) with D = diag(J), the product
// t = J D^-1 s formed as z - alpha y (z = J D^-1 r fused with v = J D^-1 p,
// y = J D^-1 v), three team barriers per iteration:
//   A: v = J phat, z = J rh            -> (rhat, v)
//   B: y = J vh; s = r - alpha v; t = z - alpha y
//                                       -> (t,s) (t,t) (rhat,s) (rhat,t) (s,s)
//   C: omega; x += alpha phat + omega D^-1 s; r = s - omega t;
//      rho' = (rhat,s) - omega (rhat,t); beta; p; phat = D^-1 p; rh = D^-1 r -> (r,r)
template <int NT, int L, int K>
__device__ KOut team_bicgstab(Team& tm, const KArgs& A, int rb, int re, double* sh, int* sh_abort) {
  const int tid = threadIdx.x;
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  EGFEM_ZERO_RED();
  if (A.x_zero) {
    for (int i = rb + tid; i < re; i += NT) {
      const double bi = A.rhs_scale * A.rhs[i];
      const double di = A.dinv[i] * bi;
      st_sh(A.x + i, 0.0);
      A.r[i] = bi;
      A.rhat[i] = bi;
      A.p[i] = bi;
      st_sh(A.phat + i, di);
      st_sh(A.rh + i, di);
      red[0] = fma(bi, bi, red[0]);
      red[1] = fma(bi, bi, red[1]);
    }
  } else {
    spmv_rows<NT, L, K, false>(A, rb, re, A.x, nullptr, [&](int i) {
      return make_double2(A.rhs[i], A.dinv[i]);
    }, [&](int i, double Jx, double, double2 q) {
      const double bi = A.rhs_scale * q.x;
      const double ri = bi - Jx;
      const double di = q.y * ri;
      A.r[i] = ri;
      A.rhat[i] = ri;
      A.p[i] = ri;
      st_sh(A.phat + i, di);
      st_sh(A.rh + i, di);
      red[0] = fma(ri, ri, red[0]);
      red[1] = fma(bi, bi, red[1]);
    });
  }
  o.abort = team_reduce<NT>(tm, 0, red, 2, sh, sh_abort);
  double rho = red[0];
  double rnorm = sqrt(red[0]);
  const double bnorm = sqrt(red[1]);
  double r0norm = rnorm;   // norm of the shadow residual rhat
  int restarts = 0;
  int slot = 1;
  int it = 0;
  if (!o.abort && bnorm == 0.0) {
    for (int i = rb + tid; i < re; i += NT) st_sh(A.x + i, 0.0);
    o.status = EGFEM_OK;
    rnorm = 0.0;
  } else {
    while (!o.abort) {
      if (!isfinite(rnorm) || !isfinite(rho)) { o.status = EGFEM_NONFINITE; break; }
      if (rnorm <= A.rtol * bnorm) { o.status = EGFEM_OK; break; }
      if (it >= A.max_iter) { o.status = EGFEM_NOT_CONVERGED; break; }
      if (fabs(rho) <= 1e-15 * r0norm * rnorm) {
        // lost bi-orthogonality: restart once from the current residual
        if (restarts++ >= 1) { o.status = EGFEM_BREAKDOWN; break; }
        EGFEM_ZERO_RED();
        for (int i = rb + tid; i < re; i += NT) {
          const double ri = A.r[i];
          A.rhat[i] = ri;
          A.p[i] = ri;
          st_sh(A.phat + i, ld_sh(A.rh + i));
          red[0] = fma(ri, ri, red[0]);
        }
        if ((o.abort = team_reduce<NT>(tm, 7, red, 1, sh, sh_abort))) break;
        rho = red[0];
        r0norm = sqrt(red[0]);   // the test above scales by the new shadow residual
        continue;
      }
      // A: v = J phat, z = J rh ; (rhat, v)
      EGFEM_ZERO_RED();
      spmv_rows<NT, L, K, true>(A, rb, re, A.phat, A.rh, [&](int i) {
        return make_double2(A.rhat[i], A.dinv[i]);
      }, [&](int i, double vi, double zi, double2 q) {
        A.v[i] = vi;
        A.z[i] = zi;
        st_sh(A.vh + i, q.y * vi);
        red[0] = fma(q.x, vi, red[0]);
      });
      if ((o.abort = team_reduce<NT>(tm, slot, red, 1, sh, sh_abort))) break;
      slot = slot % 6 + 1;
      const double rv = red[0];
      if (rv == 0.0 || !isfinite(rv)) { o.status = isfinite(rv) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
      const double alpha = rho / rv;
      // B: y = J vh ; s, t
      EGFEM_ZERO_RED();
      spmv_rows<NT, L, K, true>(A, rb, re, A.vh, nullptr, [&](int i) {
        return make_double4(A.v[i], A.r[i], A.z[i], A.rhat[i]);
      }, [&](int i, double yi, double, double4 q) {
        const double si = fma(-alpha, q.x, q.y);
        const double ti = fma(-alpha, yi, q.z);
        const double hi = q.w;
        A.s[i] = si;
        A.t[i] = ti;
        red[0] = fma(ti, si, red[0]);
        red[1] = fma(ti, ti, red[1]);
        red[2] = fma(hi, si, red[2]);
        red[3] = fma(hi, ti, red[3]);
        red[4] = fma(si, si, red[4]);
      });
      if ((o.abort = team_reduce<NT>(tm, slot, red, 5, sh, sh_abort))) break;
      slot = slot % 6 + 1;
      ++it;
      if (sqrt(red[4]) <= A.rtol * bnorm) {
        for (int i = rb + tid; i < re; i += NT) st_sh(A.x + i, fma(alpha, ld_sh(A.phat + i), ld_sh(A.x + i)));
        rnorm = sqrt(red[4]);
        o.status = EGFEM_OK;
        break;
      }
      if (red[1] == 0.0 || !isfinite(red[1])) {
        o.status = isfinite(red[1]) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE;
        break;
      }
      const double omega = red[0] / red[1];
      if (omega == 0.0) { o.status = EGFEM_BREAKDOWN; break; }
      const double rho_new = fma(-omega, red[3], red[2]);
      const double beta = (rho_new / rho) * (alpha / omega);
      rho = rho_new;
      // C: x, r, p, phat, rh ; (r, r)
      EGFEM_ZERO_RED();
      // two rows per step, every load of both before the first store (the
      // stores could alias the next row's loads, so the compiler would not
      // hoist them); the partial sum keeps the row order
      for (int i = rb + tid; i < re; i += 2 * NT) {
        const int i2 = i + NT;
        const bool two = i2 < re;
        const int j = two ? i2 : i;
        const double d1 = A.dinv[i], d2 = A.dinv[j];
        const double s1 = A.s[i], s2 = A.s[j];
        const double t1 = A.t[i], t2 = A.t[j];
        const double v1 = A.v[i], v2 = A.v[j];
        const double p1 = A.p[i], p2 = A.p[j];
        const double h1 = ld_sh(A.phat + i), h2 = ld_sh(A.phat + j);
        const double x1 = ld_sh(A.x + i), x2 = ld_sh(A.x + j);
        const double xn1 = fma(alpha, h1, fma(omega, d1 * s1, x1));
        const double xn2 = fma(alpha, h2, fma(omega, d2 * s2, x2));
        const double r1 = fma(-omega, t1, s1), r2 = fma(-omega, t2, s2);
        const double pn1 = fma(beta, fma(-omega, v1, p1), r1);
        const double pn2 = fma(beta, fma(-omega, v2, p2), r2);
        st_sh(A.x + i, xn1);
        A.r[i] = r1;
        A.p[i] = pn1;
        st_sh(A.phat + i, d1 * pn1);
        st_sh(A.rh + i, d1 * r1);
        red[0] = fma(r1, r1, red[0]);
        if (two) {
          st_sh(A.x + i2, xn2);
          A.r[i2] = r2;
          A.p[i2] = pn2;
          st_sh(A.phat + i2, d2 * pn2);
          st_sh(A.rh + i2, d2 * r2);
          red[0] = fma(r2, r2, red[0]);
        }
      }
      if ((o.abort = team_reduce<NT>(tm, slot, red, 1, sh, sh_abort))) break;
      slot = slot % 6 + 1;
      rnorm = sqrt(red[0]);
    }
  }
#undef EGFEM_ZERO_RED
  o.iters = it;
  o.rnorm = rnorm;
  o.bnorm = bnorm;
  return o;
}

// Jacobi-BiCGStab with the team's rows resident in registers: one thread per
// row (the workgroup's rows fit its threads) keeps the row's K matrix entries
// (rows hold at most K entries), its diagonal inverse and the row's vectors
// r, rhat, p, v, z, s, t, x for the whole solve.  Memory traffic per iteration
// is then the gathered vectors D^-1 p, D^-1 r, D^-1 v (agent-coherent), the
// partial sums, and x once at the end.  Same iteration as team_bicgstab, with
// (r, r) reduced together with (rhat, v) at the start of the next iteration,
// so the third synchronisation of an iteration is a plain barrier:
//   A: v = J phat, z = J rh                     -> (rhat, v), (r, r)   reduce
//      stop / restart decisions on ||r||
//   B: y = J vh; s = r - alpha v; t = z - alpha y
//                               -> (t,s) (t,t) (rhat,s) (rhat,t) (s,s) reduce
//   C: x, r, p; publish phat = D^-1 p, rh = D^-1 r                    barrier
// Row product sum_k a_k x[col_k] with the columns held as byte offsets.  The
// base pointer passes through an empty asm statement, so the compiler cannot
// hoist the per-entry 64-bit addresses out of the iteration loop (they would
// occupy two registers per entry and vector for the whole solve); the loads
// use the scalar base plus the 32-bit offset.
template <int K>
__device__ __forceinline__ double row_dot(const unsigned (&off)[K], const double (&a)[K], const double* x) {
  const char* base = reinterpret_cast<const char*>(x);
  __asm__ volatile("" : "+s"(base));
  double g[K];
#pragma unroll
  for (int k = 0; k < K; ++k) g[k] = ld_sh(reinterpret_cast<const double*>(base + off[k]));
  double acc = a[0] * g[0];
#pragma unroll
  for (int k = 1; k < K; ++k) acc = fma(a[k], g[k], acc);
  return acc;
}

// Rows wider than the K entries a thread holds in registers: entries K ..
// K + KW - 1 of the row sit in LDS, in the thread's own slice (written and
// read by that thread only, so no barrier orders them), laid out [entry][thread]
// so that a wave's accesses fall in distinct banks.  NoWide stands for KW = 0.
struct NoWide {
  static constexpr int kw = 0;
};

template <int NT, int KW, bool LX = false>
struct WideLds {
  static constexpr int kw = KW;
  double val[KW * NT];      // value (0 past the row's end and for threads without a row)
  unsigned off[KW * NT];    // column as a byte offset into a vector
  uint16_t li[KW * NT];     // part-local position of an in-block off-diagonal entry, NT otherwise
  __device__ __forceinline__ int blk(int i) const { return li[i]; }
};

// The LDS-exchange form keeps a value and a staging position per entry; the
// block position follows from the staging position (in-part off-diagonal
// entries only: the diagonal's position is the thread's own).
template <int NT, int KW>
struct WideLds<NT, KW, true> {
  static constexpr int kw = KW;
  double val[KW * NT];
  uint16_t px[KW * NT];     // staging position (own rows [0, NT), zero entry NT, ghosts above)
  __device__ __forceinline__ int blk(int i) const {
    const int p = px[i];
    return (p < NT && p != (int)threadIdx.x) ? p : NT;
  }
};

// sum over the LDS-held entries of a_e x[col_e], x gathered coherently
template <int NT, typename WX>
__device__ __forceinline__ double wide_dot(const WX& wx, const double* x, double acc) {
  if constexpr (WX::kw > 0) {
    const char* base = reinterpret_cast<const char*>(x);
    __asm__ volatile("" : "+s"(base));
    const int tid = threadIdx.x;
    double g[WX::kw];
#pragma unroll
    for (int e = 0; e < WX::kw; ++e) g[e] = ld_sh(reinterpret_cast<const double*>(base + wx.off[e * NT + tid]));
#pragma unroll
    for (int e = 0; e < WX::kw; ++e) acc = fma(wx.val[e * NT + tid], g[e], acc);
  }
  return acc;
}

// Block-Jacobi preconditioner of the register-resident BiCGStab.  The rows of
// a workgroup form one diagonal block J_b of J (the entries whose column the
// same workgroup owns), and z = M_b^-1 x approximates J_b^-1 x by a fixed
// number of Chebyshev steps with the Jacobi scaling D^-1 (Saad, Iterative
// Methods for Sparse Linear Systems, Sec. 12.3) on the interval
// [lmax / ratio, lmax] (ratio 30 unless the handle's shape sets it), lmax the
// workgroup's Gershgorin bound of
// D^-1 J_b.  The result is a fixed polynomial of D^-1 J_b applied to D^-1 x,
// i.e. a linear operator, as BiCGStab requires.  In-block products read the
// other rows' step vectors from LDS: one workgroup barrier per step and no
// traffic between workgroups.

constexpr int kMaxChebSteps = 32;

struct ChebParams {
  double theta, delta, sigma;   // centre and half width of the interval, theta / delta
  // LDS table of the step coefficients (c1, c2) of steps 1 .. kMaxChebSteps - 1:
  // they depend on the interval only, so they are formed once per solve
  const double* coef = nullptr;
};

// lmax of the workgroup: max over its rows of |d_i| (|J_ii| + sum_{in-block
// j != i} |J_ij|) (own rows only; others contribute 0).  Every thread
// returns the same value.
// Part-local positions packed two per 32-bit register (positions < 2^16), for
// kernels short of registers; indexed like the plain int array.
template <int K>
struct PackedLi {
  unsigned w[(K + 1) / 2];
  __device__ __forceinline__ int operator[](int k) const { return (int)((w[k >> 1] >> (16 * (k & 1))) & 0xffffu); }
};

// Block positions derived from staging positions (the LDS-exchange form):
// an in-part entry's staging position is its part-local position, the
// diagonal's is the thread's own, ghosts and masked entries lie at NT and
// above; only in-part off-diagonal entries belong to the block operator.
template <int NT, int K>
struct StagedLi {
  const PackedLi<K>& px;
  int tid;
  __device__ __forceinline__ int operator[](int k) const {
    const int p = px[k];
    return (p < NT && p != tid) ? p : NT;
  }
};

template <int NT, int K, typename LI, typename WX = NoWide>
__device__ ChebParams cheb_params(const LI& li, const double (&aa)[K], double ad, double d, double* lds,
                                  double ratio, const WX& wx = WX{}) {
  double g = fabs(ad);
#pragma unroll
  for (int k = 0; k < K; ++k) g += (li[k] < NT) ? fabs(aa[k]) : 0.0;
  if constexpr (WX::kw > 0) {
#pragma unroll
    for (int e = 0; e < WX::kw; ++e)
      g += (wx.blk(e * NT + threadIdx.x) < NT) ? fabs(wx.val[e * NT + threadIdx.x]) : 0.0;
  }
  g *= fabs(d);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) g = fmax(g, __shfl_xor(g, off));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = g;
  __syncthreads();
  double lmax = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) lmax = fmax(lmax, lds[w]);
  lmax = uniform(lmax);
  __syncthreads();
  if (!(lmax > 0.0) || !isfinite(lmax)) lmax = 1.0;
  const double lmin = lmax / ratio;
  ChebParams c;
  c.theta = 0.5 * (lmax + lmin);
  c.delta = 0.5 * (lmax - lmin);
  c.sigma = c.theta / c.delta;
  // rho_k = 1 / (2 sigma - rho_{k-1}) from rho_0 = 1 / sigma; step k takes
  // c1 = rho_k rho_{k-1} and c2 = 2 rho_k / delta
  __shared__ double coef[2 * kMaxChebSteps];
  if (threadIdx.x == 0) {
    double rho_old = 1.0 / c.sigma;
    coef[0] = coef[1] = 0.0;
    for (int k = 1; k < kMaxChebSteps; ++k) {
      const double rho = 1.0 / (2.0 * c.sigma - rho_old);
      coef[2 * k] = rho * rho_old;
      coef[2 * k + 1] = 2.0 * rho / c.delta;
      rho_old = rho;
    }
  }
  __syncthreads();
  c.coef = coef;
  return c;
}

// z[v] = M_b^-1 x[v] for NV vectors at once (this thread's row values).  lds
// holds two buffers of 2 (NT + 1) doubles; entry NT of each vector is 0.
// li[k] is the part-local position of an in-block off-diagonal entry, NT for
// every other entry (outside the block, the diagonal, past the row's end),
// so the K loads of a step carry no per-entry branch and are in flight
// together; ad is the row's diagonal entry.  Threads without a row (has_row
// false; whole waves at the end of a part) skip the loads.  Called by every
// thread of the workgroup.
// Workgroup barrier that orders LDS accesses only: it waits for this wave's
// LDS operations, not for its outstanding global loads, stores or atomics
// (which __syncthreads would), so global traffic issued before it stays in
// flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool LDS_ONLY>
__device__ __forceinline__ void cheb_barrier() {
  if (LDS_ONLY) lds_barrier();
  else __syncthreads();
}

template <int NT, int K, int NV, bool LDS_ONLY = false, typename LI, typename WX = NoWide>
__device__ __forceinline__ void block_cheb(const LI& li, const double (&aa)[K], double ad, double d,
                                           bool has_row, int steps, const ChebParams& c, double* lds,
                                           const double (&x)[NV], double (&z)[NV], const WX& wx = WX{}) {
  const int tid = threadIdx.x;
  double r[NV], dd[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    r[v] = x[v];
    dd[v] = d * r[v] / c.theta;
    z[v] = dd[v];
  }
  cheb_barrier<LDS_ONLY>();   // the previous call's last reads are done before this call's first writes
  for (int k = 1; k < steps; ++k) {
    double* buf = lds + (k & 1) * 2 * (NT + 1);
#pragma unroll
    for (int v = 0; v < NV; ++v) buf[v * (NT + 1) + tid] = dd[v];
    cheb_barrier<LDS_ONLY>();
    if (has_row) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = ad * dd[v];
#pragma unroll
        for (int e = 0; e < K; ++e) acc = fma(aa[e], buf[v * (NT + 1) + li[e]], acc);
        if constexpr (WX::kw > 0) {
#pragma unroll
          for (int e = 0; e < WX::kw; ++e)
            acc = fma(wx.val[e * NT + tid], buf[v * (NT + 1) + wx.blk(e * NT + tid)], acc);
        }
        r[v] -= acc;
      }
    }
    const double c1 = c.coef[2 * k], c2 = c.coef[2 * k + 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      dd[v] = fma(c1, dd[v], c2 * d * r[v]);
      z[v] += dd[v];
    }
  }
}

// LX (one workgroup per part, ghost lists in A): the products gather from
// LDS.  Before each product the workgroup stages the vector's entries of its
// own rows (each thread its row's value, which it holds) and of its ghosts
// (one coherent load per thread) in a staging vector of the Chebyshev buffer,
// laid out like the Chebyshev vectors: own rows at [0, NT), the zero entry at
// NT, ghost g at NT + 1 + g.  A row's entries then name LDS positions, and
// only the ghosts come from the coherent memory level.
template <int NT, int K, int KW = 0, bool LX = false>
__device__ KOut team_bicgstab_reg(Team& tm, const KArgs& A, int rb, int re, double* sh, int* sh_abort) {
  __shared__ double cheb_lds[4 * (NT + 1)];
  // rows of up to K + KW entries: the KW past the first K in LDS
  using WX = std::conditional_t<(KW > 0), WideLds<NT, KW, LX>, NoWide>;
  __shared__ WX wide;
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  const int i = rb + (int)threadIdx.x;
  const bool own = i < re;
  const int q = max(min(i, re - 1), 0);     // in bounds also for an empty row range
  const int row = A.rlist ? A.rlist[q] : q;
  const unsigned roff = (unsigned)row * 8u;  // byte offset of the row in a vector (n < 2^28)
  const bool bj = A.cheb_steps > 0;         // block-Jacobi preconditioner (uniform)
  // ---- the row's matrix entries (clamped in the row, zero past its end) ----
  int vi[K], li[K];
  unsigned cc[LX ? 1 : K];   // columns as byte offsets into a vector (not LX)
  int px[K];                 // staging positions (LX)
  double aa[K];
  const int beg = A.rowptr[row], end = A.rowptr[row + 1];
  bool diag[K];     // the row's diagonal entry
#pragma unroll
  for (int k = 0; k < K; ++k) {
    vi[k] = min(beg + k, end - 1);
    const int c = A.col[vi[k]];
    diag[k] = own && beg + k < end && c == row;
    if constexpr (LX) {
      const int l = A.kext[vi[k]];
      px[k] = (own && beg + k < end) ? (l >= 0 ? l : NT + 1 + (-1 - l)) : NT;
    } else {
      cc[k] = (unsigned)c * 8u;
    }
    li[k] = NT;
  }
  // the positions stay packed for the solve (two per register): the block
  // positions, or (LX) the staging positions, from which the block positions
  // follow
  PackedLi<K> lp;
#pragma unroll
  for (int k = 0; k < (K + 1) / 2; ++k) lp.w[k] = 0u;
  double ad = 0.0;   // diagonal entry (block-Jacobi)
  if (bj) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int l = A.kloc[vi[k]];
      const bool offd = own && beg + k < end && !diag[k];
      li[k] = (offd && l >= 0) ? l : NT;
    }
  }
  if (A.perm) {
#pragma unroll
    for (int k = 0; k < K; ++k) vi[k] = A.perm[vi[k]];
  }
  // row values, D^-1 and the right-hand side with agent-coherent loads: in a
  // batched launch other workgroups of the team emitted them
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double w = ld_sh(A.val + vi[k]);
    aa[k] = (own && beg + k < end) ? w : 0.0;
  }
  const double d = ld_sh(A.dinv + row);
  const double b = A.rhs_scale * ld_sh(A.rhs + row);
  if constexpr (KW > 0) {
    // entries K .. K + KW - 1 (clamped in the row, zero past its end) to LDS
#pragma unroll
    for (int e = 0; e < KW; ++e) {
      int sk = min(beg + K + e, end - 1);
      const int ck = A.col[sk];
      const bool in = own && beg + K + e < end;
      int l = NT;
      if (bj) {
        const int kl = A.kloc[sk];
        if (in && ck != row && kl >= 0) l = kl;
      }
      unsigned wofs = (unsigned)ck * 8u;
      if constexpr (LX) {
        const int x = A.kext[sk];
        wofs = in ? (unsigned)(x >= 0 ? x : NT + 1 + (-1 - x)) : (unsigned)NT;
      }
      if (A.perm) sk = A.perm[sk];
      const double w = ld_sh(A.val + sk);
      const double wv = in ? w : 0.0;
      if (bj && in && ck == row) ad = wv;
      wide.val[e * NT + threadIdx.x] = wv;
      if constexpr (LX) {
        wide.px[e * NT + threadIdx.x] = (uint16_t)wofs;
      } else {
        wide.off[e * NT + threadIdx.x] = wofs;
        wide.li[e * NT + threadIdx.x] = (uint16_t)l;
      }
    }
  }
  ChebParams cp{1.0, 1.0, 1.0};
  if (bj) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (diag[k]) ad = aa[k];
    cp = cheb_params<NT, K>(li, aa, ad, d, cheb_lds, A.cheb_ratio, wide);
    if constexpr (!LX) {
#pragma unroll
      for (int k = 0; k < K; ++k) lp.w[k >> 1] |= (unsigned)li[k] << (16 * (k & 1));
    }
    if (threadIdx.x < 4) cheb_lds[(threadIdx.x >> 1) * 2 * (NT + 1) + (threadIdx.x & 1) * (NT + 1) + NT] = 0.0;
  }
  if constexpr (LX) {
#pragma unroll
    for (int k = 0; k < K; ++k) lp.w[k >> 1] |= (unsigned)px[k] << (16 * (k & 1));
  }
  const StagedLi<NT, K> sli{lp, (int)threadIdx.x};
  // M^-1 of this thread's row values: D^-1 or the block-Jacobi operator
  auto prec1 = [&](double x1) -> double {
    if (!bj) return d * x1;
    const double xs[1] = {x1};
    double zs[1];
    if constexpr (LX) block_cheb<NT, K, 1>(sli, aa, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs, wide);
    else block_cheb<NT, K, 1>(lp, aa, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs, wide);
    return zs[0];
  };
  // ---- LDS-exchange products (LX) -----------------------------------------
  // this part's ghosts: thread t < ng stages ghost t
  int ng = 0;
  unsigned gofs = 0u;
  if constexpr (LX) {
    const int g0 = A.gptr[blockIdx.x];
    ng = A.gptr[blockIdx.x + 1] - g0;
    gofs = (unsigned)A.gcol[g0 + min((int)threadIdx.x, max(ng - 1, 0))] * 8u;
  }
  // S[own position] = this thread's row value, S[NT + 1 + t] = ghost t of vec
  // (the zero entry S[NT] is never written: it is the Chebyshev buffer's)
  auto stage = [&](double* S, double own_val, const double* vec) {
    S[threadIdx.x] = own_val;
    if ((int)threadIdx.x < ng) S[NT + 1 + threadIdx.x] = ld_sh_at(vec, gofs);
  };
  auto lds_dot = [&](const double* S) -> double {
    double acc = aa[0] * S[lp[0]];
#pragma unroll
    for (int k = 1; k < K; ++k) acc = fma(aa[k], S[lp[k]], acc);
    if constexpr (KW > 0 && LX) {
#pragma unroll
      for (int e = 0; e < KW; ++e) acc = fma(wide.val[e * NT + threadIdx.x], S[wide.px[e * NT + threadIdx.x]], acc);
    }
    return acc;
  };
  double* const S0 = cheb_lds;                 // staging vectors: the two Chebyshev buffers
  double* const S1 = cheb_lds + 2 * (NT + 1);
  // ---- r = b - J x ; rhat = p = r ; publish M^-1 r --------------------------
  double x = 0.0, r = b;
  if (!A.x_zero) {
    // once per solve: the columns from the matrix (LX rows name LDS positions)
    double g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = A.x[A.col[min(beg + k, end - 1)]];
    x = A.x[row];
    double acc = aa[0] * g[0];
#pragma unroll
    for (int k = 1; k < K; ++k) acc = fma(aa[k], g[k], acc);
    if constexpr (KW > 0) {
#pragma unroll
      for (int e = 0; e < KW; ++e)
        acc = fma(wide.val[e * NT + threadIdx.x], A.x[A.col[min(beg + K + e, end - 1)]], acc);
    }
    r = b - acc;
  }
  if (!own) r = 0.0;
  // the iterate x is updated once per iteration: it lives in memory (this
  // thread's row, written coherently: inside a batched launch other workgroups
  // of the team gather it before the launch ends), not in registers
  if (own) st_sh_at(A.x, roff, x);
  // the shadow residual r^ is read three times per iteration and written only
  // at a restart: it lives in memory (this thread's row), not in registers
  // (threads without a row alias the part's last row: only owners write)
  if (own) st_at(A.rhat, roff, r);
  // the direction p itself is not kept: its preconditioned form follows
  // from the recurrence below
  double v = 0.0, z = 0.0, sv = 0.0, tv = 0.0;
  // this row's entries of the published vectors: M^-1 p, M^-1 r, M^-1 v
  double ph = prec1(r), rhh = ph, vhh = 0.0;
  EGFEM_ZERO_RED();
  if (own) {
    st_sh_at(A.phat, roff, ph);
    st_sh_at(A.rh, roff, rhh);
    red[1] = b * b;
  }
  if ((o.abort = team_reduce<NT>(tm, 0, red, 2, sh, sh_abort))) return o;
  const double bnorm = sqrt(red[1]);
  o.bnorm = bnorm;
  if (bnorm == 0.0) {
    if (own) st_sh_at(A.x, roff, 0.0);
    o.status = EGFEM_OK;
    return o;
  }
  double rho = 0.0, rnorm = 0.0, r0norm = -1.0;
  int restarts = 0, slot = 1, it = 0;
  while (true) {
    // A: v = J phat, z = J rh ; (rhat, v), (r, r)
    if constexpr (LX) {
      __syncthreads();   // the last reads of the Chebyshev buffers are done
      stage(S0, ph, A.phat);
      stage(S1, rhh, A.rh);
      __syncthreads();
      v = lds_dot(S0);
      z = lds_dot(S1);
    } else {
      v = wide_dot<NT>(wide, A.phat, row_dot<K>(cc, aa, A.phat));
      z = wide_dot<NT>(wide, A.rh, row_dot<K>(cc, aa, A.rh));
    }
    vhh = prec1(v);
    EGFEM_ZERO_RED();
    if (own) {
      st_sh_at(A.vh, roff, vhh);
      red[0] = ld_at(A.rhat, roff) * v;
      red[1] = r * r;
    }
    if ((o.abort = team_reduce<NT>(tm, slot, red, 2, sh, sh_abort))) break;
    slot = slot % 6 + 1;
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
      // lost bi-orthogonality: restart once from the current residual
      // (p = r, so M^-1 p is the published M^-1 r)
      if (restarts++ >= 1) { o.status = EGFEM_BREAKDOWN; break; }
      if (own) st_at(A.rhat, roff, r);
      ph = rhh;
      if (own) st_sh_at(A.phat, roff, ph);
      rho = red[1];
      r0norm = rnorm;   // the test above scales by the new shadow residual
      if ((o.abort = team_barrier(tm, sh_abort))) break;
      continue;
    }
    if (rv == 0.0 || !isfinite(rv)) { o.status = isfinite(rv) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE; break; }
    const double alpha = rho / rv;
    // B: y = J vh ; s, t
    {
      double y;
      if constexpr (LX) {
        __syncthreads();
        stage(S0, vhh, A.vh);
        __syncthreads();
        y = lds_dot(S0);
      } else {
        y = wide_dot<NT>(wide, A.vh, row_dot<K>(cc, aa, A.vh));
      }
      sv = fma(-alpha, v, r);
      tv = fma(-alpha, y, z);
      EGFEM_ZERO_RED();
      if (own) {
        red[0] = tv * sv;
        red[1] = tv * tv;
        const double rhv = ld_at(A.rhat, roff);
        red[2] = rhv * sv;
        red[3] = rhv * tv;
        red[4] = sv * sv;
      }
    }
    if ((o.abort = team_reduce<NT>(tm, slot, red, 5, sh, sh_abort))) break;
    slot = slot % 6 + 1;
    ++it;
    if (sqrt(red[4]) <= A.rtol * bnorm) {
      if (own) st_sh_at(A.x, roff, fma(alpha, ph, ld_sh_at(A.x, roff)));
      rnorm = sqrt(red[4]);
      o.status = EGFEM_OK;
      break;
    }
    if (red[1] == 0.0 || !isfinite(red[1])) {
      o.status = isfinite(red[1]) ? EGFEM_BREAKDOWN : EGFEM_NONFINITE;
      break;
    }
    const double omega = red[0] / red[1];
    if (omega == 0.0) { o.status = EGFEM_BREAKDOWN; break; }
    const double rho_new = fma(-omega, red[3], red[2]);
    const double beta = (rho_new / rho) * (alpha / omega);
    rho = rho_new;
    // C: x, r ; publish M^-1 p, M^-1 r  (M^-1 s = M^-1 r - alpha M^-1 v).
    // M^-1 is linear, so p = r + beta (p - omega v) gives
    // M^-1 p = M^-1 r + beta (M^-1 p - omega M^-1 v): one application per
    // iteration (M^-1 r) besides M^-1 v
    if (own) st_sh_at(A.x, roff, fma(alpha, ph, fma(omega, bj ? fma(-alpha, vhh, rhh) : d * sv, ld_sh_at(A.x, roff))));
    r = fma(-omega, tv, sv);
    rhh = prec1(r);
    ph = fma(beta, fma(-omega, vhh, ph), rhh);
    if (own) {
      st_sh_at(A.phat, roff, ph);
      st_sh_at(A.rh, roff, rhh);
    }
    // phase A gathers M^-1 p and M^-1 r of neighbouring rows only; the two
    // team reductions before the next overwrite keep the reads ahead of it
    if ((o.abort = team_neighbor_sync(tm, sh_abort))) break;
  }
#undef EGFEM_ZERO_RED

  o.iters = it;
  o.rnorm = rnorm;
  return o;
}

// Preconditioned conjugate gradients for a symmetric positive definite J (the
// Picard matrix), in the single-reduction arrangement of Chronopoulos and
// Gear: with u = M^-1 r and w = J u, the scalars gamma = (r, u) and
// delta = (w, u) give beta = gamma / gamma_prev and
// alpha = gamma / (delta - beta gamma / alpha_prev), and s = J p is kept by the
// recurrence s = w + beta s.  Per iteration: one product (gathering M^-1 r),
// one reduction of (r, u), (w, u), (r, r), one barrier after publishing M^-1 r.
// Stops when ||r|| <= rtol ||r0|| (rel_r0) or rtol ||b||.
// Register-resident form: one thread per row (rows fit the workgroup's
// threads, at most K entries), matrix row, D^-1 and the row's x, r, p, s in
// registers for the whole solve; M is D (Jacobi) or, on a compact partition,
// the block-Jacobi operator of block_cheb.
template <int NT, int K>
__device__ KOut team_pcg_reg(Team& tm, const KArgs& A, int rb, int re, double* sh, int* sh_abort) {
  __shared__ double cheb_lds[4 * (NT + 1)];
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  const int i = rb + (int)threadIdx.x;
  const bool own = i < re;
  const int q = max(min(i, re - 1), 0);
  const int row = A.rlist ? A.rlist[q] : q;
  const bool bj = A.cheb_steps > 0;         // block-Jacobi preconditioner (uniform)
  int vi[K], li[K];
  unsigned cc[K];
  double aa[K];
  const int beg = A.rowptr[row], end = A.rowptr[row + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    vi[k] = min(beg + k, end - 1);
    cc[k] = (unsigned)A.col[vi[k]] * 8u;
    li[k] = NT;
  }
  double ad = 0.0;   // diagonal entry (block-Jacobi)
  if (bj) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int l = A.kloc[vi[k]];
      const bool offd = own && beg + k < end && (int)(cc[k] / 8u) != row;
      li[k] = (offd && l >= 0) ? l : NT;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double w = A.val[vi[k]];
    aa[k] = (own && beg + k < end) ? w : 0.0;
  }
  const double d = A.dinv[row];
  const double b = A.rhs_scale * A.rhs[row];
  ChebParams cp{1.0, 1.0, 1.0};
  if (bj) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (own && beg + k < end && (int)(cc[k] / 8u) == row) ad = aa[k];
    cp = cheb_params<NT, K>(li, aa, ad, d, cheb_lds, A.cheb_ratio);
    if (threadIdx.x < 4) cheb_lds[(threadIdx.x >> 1) * 2 * (NT + 1) + (threadIdx.x & 1) * (NT + 1) + NT] = 0.0;
  }
  // M^-1 of this thread's row value: D^-1 or the block-Jacobi operator (SPD
  // for an SPD J: the Chebyshev polynomial is positive on (0, lmax])
  auto prec1 = [&](double x1) -> double {
    if (!bj) return d * x1;
    const double xs[1] = {x1};
    double zs[1];
    block_cheb<NT, K, 1>(li, aa, ad, d, own, A.cheb_steps, cp, cheb_lds, xs, zs);
    return zs[0];
  };
  double x = 0.0, r = b;
  if (!A.x_zero) {
    double g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = A.x[cc[k] / 8u];
    x = A.x[row];
    double acc = aa[0] * g[0];
#pragma unroll
    for (int k = 1; k < K; ++k) acc = fma(aa[k], g[k], acc);
    r = b - acc;
  }
  if (!own) r = 0.0;
  double u = prec1(r), p = 0.0, s = 0.0;
  EGFEM_ZERO_RED();
  if (own) {
    st_sh(A.phat + row, u);
    red[0] = b * b;
  }
  if ((o.abort = team_reduce<NT>(tm, 0, red, 1, sh, sh_abort))) return o;
  const double bnorm = sqrt(red[0]);
  double ref = bnorm, gamma_prev = 0.0, alpha_prev = 0.0, rnorm = 0.0;
  int slot = 1, it = 0;
  while (true) {
    const double w = row_dot<K>(cc, aa, A.phat);
    EGFEM_ZERO_RED();
    if (own) {
      red[0] = r * u;
      red[1] = w * u;
      red[2] = r * r;
    }
    if ((o.abort = team_reduce<NT>(tm, slot, red, 3, sh, sh_abort))) break;
    slot = slot % 6 + 1;
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
    s = fma(beta, s, w);
    x = fma(alpha, p, x);
    r = fma(-alpha, s, r);
    u = prec1(r);
    if (own) st_sh(A.phat + row, u);
    gamma_prev = gamma;
    alpha_prev = alpha;
    ++it;
    // the next product gathers M^-1 r of neighbouring rows; the reduction
    // before the next overwrite keeps every read ahead of it
    if ((o.abort = team_neighbor_sync(tm, sh_abort))) break;
  }
#undef EGFEM_ZERO_RED
  if (!o.abort && own) A.x[row] = x;
  o.iters = it;
  o.rnorm = rnorm;
  o.bnorm = ref;
  return o;
}

// Streaming form of the same iteration (any number of rows per workgroup):
// the row vectors r, p, s, x and w live in memory, the product reads J.
template <int NT, int L, int K>
__device__ KOut team_pcg(Team& tm, const KArgs& A, int rb, int re, double* sh, int* sh_abort) {
  const int tid = threadIdx.x;
  double red[kMaxRed];
  KOut o{EGFEM_NOT_CONVERGED, 0, 0.0, 0.0, false};
#define EGFEM_ZERO_RED() for (int q_ = 0; q_ < kMaxRed; ++q_) red[q_] = 0.0
  EGFEM_ZERO_RED();
  if (A.x_zero) {
    for (int i = rb + tid; i < re; i += NT) {
      const double bi = A.rhs_scale * A.rhs[i];
      A.x[i] = 0.0;
      A.r[i] = bi;
      A.p[i] = 0.0;
      A.s[i] = 0.0;
      st_sh(A.phat + i, A.dinv[i] * bi);
      red[0] = fma(bi, bi, red[0]);
    }
  } else {
    spmv_rows<NT, L, K, false>(A, rb, re, A.x, nullptr, [&](int i) {
      return make_double2(A.rhs[i], A.dinv[i]);
    }, [&](int i, double Jx, double, double2 q) {
      const double bi = A.rhs_scale * q.x;
      const double ri = bi - Jx;
      A.r[i] = ri;
      A.p[i] = 0.0;
      A.s[i] = 0.0;
      st_sh(A.phat + i, q.y * ri);
      red[0] = fma(bi, bi, red[0]);
    });
  }
  if ((o.abort = team_reduce<NT>(tm, 0, red, 1, sh, sh_abort))) return o;
  const double bnorm = sqrt(red[0]);
  double ref = bnorm, gamma_prev = 0.0, alpha_prev = 0.0, rnorm = 0.0;
  int slot = 1, it = 0;
  while (true) {
    EGFEM_ZERO_RED();
    spmv_rows<NT, L, K, true>(A, rb, re, A.phat, nullptr, [&](int i) {
      return make_double2(A.r[i], A.dinv[i]);
    }, [&](int i, double wi, double, double2 q) {
      const double ui = q.y * q.x;
      A.v[i] = wi;
      red[0] = fma(q.x, ui, red[0]);
      red[1] = fma(wi, ui, red[1]);
      red[2] = fma(q.x, q.x, red[2]);
    });
    if ((o.abort = team_reduce<NT>(tm, slot, red, 3, sh, sh_abort))) break;
    slot = slot % 6 + 1;
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
    for (int i = rb + tid; i < re; i += NT) {
      const double di = A.dinv[i], ri = A.r[i], wi = A.v[i];
      const double pi = fma(beta, A.p[i], di * ri);
      const double si = fma(beta, A.s[i], wi);
      const double xi = fma(alpha, pi, A.x[i]);
      const double rn = fma(-alpha, si, ri);
      A.p[i] = pi;
      A.s[i] = si;
      A.x[i] = xi;
      A.r[i] = rn;
      st_sh(A.phat + i, di * rn);
    }
    gamma_prev = gamma;
    alpha_prev = alpha;
    ++it;
    if ((o.abort = team_neighbor_sync(tm, sh_abort))) break;
  }
#undef EGFEM_ZERO_RED
  o.iters = it;
  o.rnorm = rnorm;
  o.bnorm = ref;
  return o;
}

}  // namespace dev
}  // namespace egfem
