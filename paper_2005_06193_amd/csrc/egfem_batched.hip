// Batched EGFEM Newton: many independent instances in ONE persistent
// cooperative launch.  Instance m is owned by a team of consecutive
// workgroups; each team member owns a contiguous range of the instance's row
// blocks (hence a contiguous range of rows), so Jacobian rows, residual rows
// and Krylov rows of a member coincide and only gathered vectors (u, the
// Newton correction, the preconditioned Krylov vectors) cross workgroups,
// through agent-coherent accesses.  The whole damped Newton loop -- residual
// with fused pointwise update, Jacobian emission, BiCGStab, line search,
// convergence test -- runs on the device with team-local barriers.
//
// Two plan kinds.  Streaming teams: every instance has its team for the whole
// launch and its members stream their rows through the Jacobi BiCGStab.
// Scheduled resident teams: a member owns at most one row per thread, so the
// Krylov solve is the register-resident block-Jacobi BiCGStab (the member's
// rows are its block); the teams that this needs exceed the co-resident
// workgroups, so the host packs the instances into the resident workgroups in
// space and time (list scheduling on an estimated duration), and every
// workgroup runs its own list of (instance, rank) in start order.  A team
// forms when its members reach the instance's first team barrier; since every
// workgroup takes its instances in the order of their start times, no wait can
// close a cycle.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "egfem_device.h"

namespace egfem {

dev::TensorView view_of(const egfem_tensor_s* T);

namespace {

// status, iters, krylov, backtracks, res0, res, then per step: residual, Krylov
// iterations, Krylov status, Krylov relative residual
constexpr int kStatsWords = 6 + 4 * EGFEM_HIST;

struct Inst {
  dev::TensorView tv;
  const double* a0;
  double a0c;
  const double* load;
  const uint8_t* dir;
  int addK;
  double* u;          // caller buffer: guess in / solution out
  double* utry;       // second iterate buffer
  double* F;
  double* jval;
  double* dinv;
  dev::KArgs K;       // matrix = jval, rhs = F (scale -1), x = Newton correction
  const int32_t* wgblk;   // [team_size + 1] row-block range of every member
  // scheduled resident teams: member q's Krylov rows are K.rlist[kr[q], kr[q+1])
  // (a part of the compact partition); nbr its neighbour list, or null
  const int32_t* kr;
  const int32_t* nbr;
  unsigned* ctrl;
  double* red;
  double* stats;      // [kStatsWords]
  int team_first;
  int team_size;
};

struct BatchOpts {
  double tol;
  int max_newton;
  int max_krylov;
  double krylov_rtol;
  int forcing;
  double eta_max;
  int max_backtracks;
  int zero_init;
};

// Eisenstat-Walker choice 2 with the safeguards of the host driver.
__device__ double ew_forcing(int k, double nF, double nF_prev, double eta_prev, double eta_max,
                             double tol_abs) {
  double eta;
  if (k == 0) {
    eta = eta_max;
  } else {
    eta = 0.9 * (nF / nF_prev) * (nF / nF_prev);
    const double guard = 0.9 * eta_prev * eta_prev;
    if (guard > 0.1) eta = fmax(eta, guard);
    eta = fmin(eta, eta_max);
  }
  eta = fmax(eta, 0.5 * tol_abs / nF);
  return fmin(eta, eta_max);
}

// The damped Newton loop of instance I by team member tm (row blocks [b0, b1)).
// RES: the Krylov solve is the register-resident block-Jacobi BiCGStab (the
// member's rows fit its threads); otherwise the streaming Jacobi BiCGStab.
template <int NT, int RS, bool RES>
__device__ void newton_team(const Inst& I, dev::Team& tm, int b0, int b1, const BatchOpts& O,
                            dev::RowBlockLds& lds, double* sh, int& sh_abort) {
  const int rb = I.tv.blk_row[b0], re = I.tv.blk_row[b1];
  const int tid = threadIdx.x;
  const double* kval = I.addK ? I.tv.kval : nullptr;
  double red[dev::kMaxRed];
  int nslot = 8;
  bool abort = false;

  // initial iterate (Dirichlet entries 0), published to the team
  for (int i = rb + tid; i < re; i += NT) {
    double ui = O.zero_init ? 0.0 : I.u[i];
    if (I.dir && I.dir[i]) ui = 0.0;
    dev::st_sh(I.u + i, ui);
  }
  abort = dev::team_barrier(tm, &sh_abort);
  double* ucur = I.u;
  double* unext = I.utry;

  // residual at the initial iterate
  double sq = 0.0;
  if (!abort)
    dev::rowblocks_action_pipelined<NT, true, true>(I.tv, b0, b1, ucur, nullptr, 0.0, I.a0, I.a0c, I.load,
                                                    I.dir, kval, I.F, nullptr, sq, lds);
  for (int q = 0; q < dev::kMaxRed; ++q) red[q] = 0.0;
  red[0] = sq;
  if (!abort) abort = dev::team_reduce<NT>(tm, nslot, red, 1, sh, &sh_abort);
  nslot = 17 - nslot;
  const double nF0 = sqrt(red[0]);
  double nF = nF0, nF_prev = nF0, eta = O.eta_max;
  int status = EGFEM_NOT_CONVERGED;
  if (!isfinite(nF0)) status = EGFEM_NONFINITE;
  else if (nF0 == 0.0) status = EGFEM_OK;
  int k = 0, kry = 0, backtracks = 0;
  double* st = I.stats;
  const bool writer = (tm.rank == 0 && tid == 0);
  // histories start cleared: a replay must not report the previous run's steps
  if (tm.rank == 0)
    for (int q = 6 + tid; q < kStatsWords; q += NT) st[q] = 0.0;

  while (!abort && status == EGFEM_NOT_CONVERGED) {
    if (nF <= O.tol * nF0) { status = EGFEM_OK; break; }
    if (k >= O.max_newton) break;
    // Jacobian emission for the member's own rows
    for (int b = b0; b < b1; ++b)
      dev::rowblock_jacobian<NT, true>(I.tv, b, ucur, nullptr, I.a0, I.a0c, 1, nullptr, 1, kval, I.dir,
                                       I.jval, I.dinv, lds);
    const double rtol = O.forcing ? ew_forcing(k, nF, nF_prev, eta, O.eta_max, O.tol * nF0) : O.krylov_rtol;
    eta = rtol;
    dev::KArgs KA = I.K;
    KA.rtol = rtol;
    KA.max_iter = O.max_krylov;
    dev::KOut ko;
    if constexpr (RES) {
      // the member's Krylov rows are its part of the compact partition: rows
      // whose Jacobian, D^-1 and residual other members emitted
      if ((abort = dev::team_barrier(tm, &sh_abort))) break;
      ko = dev::team_bicgstab_reg<NT, kResidentRow>(tm, KA, I.kr[tm.rank], I.kr[tm.rank + 1], sh, &sh_abort);
    } else {
      ko = dev::team_bicgstab<NT, row_L(RS), row_K(RS)>(tm, KA, rb, re, sh, &sh_abort);
    }
    if ((abort = ko.abort)) break;
    kry += ko.iters;
    if (writer && k < EGFEM_HIST) {
      st[6 + EGFEM_HIST + k] = (double)ko.iters;
      st[6 + 2 * EGFEM_HIST + k] = (double)ko.status;
      st[6 + 3 * EGFEM_HIST + k] = ko.bnorm > 0.0 ? ko.rnorm / ko.bnorm : 0.0;
    }
    if (ko.status == EGFEM_NONFINITE) { status = EGFEM_NONFINITE; break; }
    if ((abort = dev::team_barrier(tm, &sh_abort))) break;   // correction visible to the team
    // damped update with the residual of the trial iterate
    double alpha = 1.0, nFt = 0.0;
    bool accepted = false;
    for (int bt = 0; bt <= O.max_backtracks; ++bt) {
      sq = 0.0;
      dev::rowblocks_action_pipelined<NT, true, true>(I.tv, b0, b1, ucur, KA.x, alpha, I.a0, I.a0c, I.load,
                                                      I.dir, kval, I.F, unext, sq, lds);
      for (int q = 0; q < dev::kMaxRed; ++q) red[q] = 0.0;
      red[0] = sq;
      if ((abort = dev::team_reduce<NT>(tm, nslot, red, 1, sh, &sh_abort))) break;
      nslot = 17 - nslot;
      nFt = sqrt(red[0]);
      if (isfinite(nFt) && nFt <= (1.0 - 1e-4 * alpha) * nF) { accepted = true; break; }
      alpha *= 0.5;
      ++backtracks;
    }
    if (abort) break;
    if (!accepted) { status = EGFEM_STAGNATED; break; }
    double* tmp = ucur;
    ucur = unext;
    unext = tmp;
    nF_prev = nF;
    nF = nFt;
    if (writer && k < EGFEM_HIST) st[6 + k] = nF;
    ++k;
  }
  if (!abort && status == EGFEM_NOT_CONVERGED && nF <= O.tol * nF0) status = EGFEM_OK;
  // the solution lives in the caller's buffer
  if (!abort && ucur != I.u)
    for (int i = rb + tid; i < re; i += NT) I.u[i] = dev::ld_sh(ucur + i);
  if (writer) {
    st[0] = abort ? (double)EGFEM_ERR_HIP : (double)status;
    st[1] = (double)k;
    st[2] = (double)kry;
    st[3] = (double)backtracks;
    st[4] = nF0;
    st[5] = nF;
  }
}

template <int NT, int RS>
__global__ __launch_bounds__(NT) void k_newton_batched(const Inst* __restrict__ insts,
                                                       const int32_t* __restrict__ wg2inst, BatchOpts O) {
  __shared__ dev::RowBlockLds lds;
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_abort;
  const Inst& I = insts[wg2inst[blockIdx.x]];
  dev::Team tm{blockIdx.x - (unsigned)I.team_first, (unsigned)I.team_size, I.ctrl, I.red, 0u};
  newton_team<NT, RS, false>(I, tm, I.wgblk[tm.rank], I.wgblk[tm.rank + 1], O, lds, sh, sh_abort);
}

// Scheduled resident teams: workgroup w runs the (instance, rank) pairs
// list[ptr[w], ptr[w + 1]) in order.
template <int NT>
__global__ __launch_bounds__(NT) void k_newton_sched(const Inst* __restrict__ insts,
                                                     const int32_t* __restrict__ ptr,
                                                     const int2* __restrict__ list, BatchOpts O) {
  __shared__ dev::RowBlockLds lds;
  __shared__ double sh[dev::kShWords<NT>];
  __shared__ int sh_abort;
  for (int t = ptr[blockIdx.x]; t < ptr[blockIdx.x + 1]; ++t) {
    const int2 e = list[t];
    const Inst& I = insts[e.x];
    dev::Team tm{(unsigned)e.y, (unsigned)I.team_size, I.ctrl, I.red, 0u};
    if (I.nbr) tm.nbr = I.nbr + (size_t)e.y * (dev::kMaxNbr + 1);
    newton_team<NT, 0, true>(I, tm, I.wgblk[e.y], I.wgblk[e.y + 1], O, lds, sh, sh_abort);
  }
}

template <int NT, int RS>
hipError_t launch_NL(const Inst* insts, const int32_t* wg2inst, const BatchOpts& O, unsigned G,
                     hipStream_t st) {
  void* args[] = {(void*)&insts, (void*)&wg2inst, (void*)&O};
  return hipLaunchCooperativeKernel((const void*)k_newton_batched<NT, RS>, dim3(G), dim3(NT), args, 0, st);
}

template <int NT, int RS>
int cap_NL() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_newton_batched<NT, RS>, NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

template <int NT>
hipError_t launch_sched(const Inst* insts, const int32_t* ptr, const int2* list, const BatchOpts& O, unsigned G,
                        hipStream_t st) {
  void* args[] = {(void*)&insts, (void*)&ptr, (void*)&list, (void*)&O};
  return hipLaunchCooperativeKernel((const void*)k_newton_sched<NT>, dim3(G), dim3(NT), args, 0, st);
}

template <int NT>
int cap_sched() {
  int dev = 0, per_cu = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_newton_sched<NT>, NT, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

template <int NT>
hipError_t launch_T(int L, const Inst* insts, const int32_t* wg2inst, const BatchOpts& O, unsigned G,
                    hipStream_t st) {
  switch (L) {
    case 0: return launch_NL<NT, 0>(insts, wg2inst, O, G, st);
    case 1: return launch_NL<NT, 1>(insts, wg2inst, O, G, st);
    case 2: return launch_NL<NT, 2>(insts, wg2inst, O, G, st);
    case 3: return launch_NL<NT, 3>(insts, wg2inst, O, G, st);
    case 4: return launch_NL<NT, 4>(insts, wg2inst, O, G, st);
    case 5: return launch_NL<NT, 5>(insts, wg2inst, O, G, st);
    case 6: return launch_NL<NT, 6>(insts, wg2inst, O, G, st);
    case 7: return launch_NL<NT, 7>(insts, wg2inst, O, G, st);
    default: return launch_NL<NT, 8>(insts, wg2inst, O, G, st);
  }
}

template <int NT>
int cap_T(int L) {
  switch (L) {
    case 0: return cap_NL<NT, 0>();
    case 1: return cap_NL<NT, 1>();
    case 2: return cap_NL<NT, 2>();
    case 3: return cap_NL<NT, 3>();
    case 4: return cap_NL<NT, 4>();
    case 5: return cap_NL<NT, 5>();
    case 6: return cap_NL<NT, 6>();
    case 7: return cap_NL<NT, 7>();
    default: return cap_NL<NT, 8>();
  }
}

}  // namespace
}  // namespace egfem

struct egfem_batch_s {
  int count = 0;
  int kind = 0;       // 0 streaming teams, 1 scheduled resident teams
  int NT = 512;
  int L = 4;
  int G = 0;
  std::vector<egfem_tensor_t> Ts;
  std::vector<int> team;
  egfem::BatchOpts opts{};
  egfem::Inst* d_insts = nullptr;
  int32_t* d_wg2inst = nullptr;
  int32_t* d_wgblk = nullptr;
  unsigned* d_ctrl = nullptr;
  double* d_red = nullptr;
  double* d_stats = nullptr;
  double* h_stats = nullptr;
  size_t ctrl_words = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_zero_init = -1;
  hipStream_t cap_stream = nullptr;   // capture stream owned by the plan (default priority)
  // scheduled resident teams: per-workgroup (instance, rank) lists, part-local
  // column positions of every instance's slots
  int32_t* d_sched_ptr = nullptr;
  int2* d_sched_list = nullptr;
  int16_t* d_kloc = nullptr;
  int32_t* d_kr = nullptr;      // every instance's part offsets
  int32_t* d_rlist = nullptr;   // every instance's part rows
  int32_t* d_nbr = nullptr;     // every instance's neighbour lists
  double makespan = 0.0;   // of the schedule, in the duration model's units
};

namespace {

void free_batch(egfem_batch_s* B) {
  if (!B) return;
  if (B->exec) hipGraphExecDestroy(B->exec);
  if (B->graph) hipGraphDestroy(B->graph);
  if (B->cap_stream) hipStreamDestroy(B->cap_stream);
  if (B->d_insts) hipFree(B->d_insts);
  if (B->d_wg2inst) hipFree(B->d_wg2inst);
  if (B->d_wgblk) hipFree(B->d_wgblk);
  if (B->d_ctrl) hipFree(B->d_ctrl);
  if (B->d_red) hipFree(B->d_red);
  if (B->d_stats) hipFree(B->d_stats);
  if (B->h_stats) hipHostFree(B->h_stats);
  if (B->d_sched_ptr) hipFree(B->d_sched_ptr);
  if (B->d_sched_list) hipFree(B->d_sched_list);
  if (B->d_kloc) hipFree(B->d_kloc);
  if (B->d_kr) hipFree(B->d_kr);
  if (B->d_rlist) hipFree(B->d_rlist);
  if (B->d_nbr) hipFree(B->d_nbr);
  delete B;
}

// Newton options of a batch (defaults where o is null), validated.
int batch_opts(const egfem_newton_opts* o, egfem_newton_opts* out) {
  using namespace egfem;
  egfem_newton_opts_default(out);
  if (o) *out = *o;
  if (!(out->tol >= 0.0) || out->max_newton < 0 || out->max_krylov < 1 || !(out->krylov_rtol > 0.0) ||
      !(out->eta_max > 0.0 && out->eta_max < 1.0) || out->max_backtracks < 0)
    return fail(EGFEM_ERR_ARG, "invalid Newton options");
  return EGFEM_OK;
}

int batch_handles(int count, const egfem_tensor_t* Ts, double* const* us) {
  using namespace egfem;
  for (int m = 0; m < count; ++m) {
    if (!Ts[m] || !us[m]) return fail(EGFEM_ERR_ARG, "null handle or solution buffer");
    if (Ts[m]->w2) return fail(EGFEM_ERR_ARG, "the batched form is not available for handles with W_h != P1");
    for (int q = 0; q < m; ++q)
      if (Ts[q] == Ts[m]) return fail(EGFEM_ERR_ARG, "a handle appears twice in the batch");
  }
  return EGFEM_OK;
}

// Descriptor of instance m (its handle's workspace holds the Newton and
// Krylov vectors); team and buffer pointers are set by the caller.
void fill_inst(egfem::Inst& I, egfem_tensor_s* T, const egfem_problem& p, double* u,
               const egfem_newton_opts& opts) {
  using namespace egfem;
  Workspace& W = T->ws;
  I.tv = view_of(T);
  I.a0 = p.a0;
  I.a0c = p.a0_const;
  I.load = p.load;
  I.dir = p.dirichlet;
  I.addK = p.add_stiffness;
  I.u = u;
  I.utry = W.utry;
  I.F = W.F;
  I.jval = W.jval;
  I.dinv = W.dinv;
  dev::KArgs& K = I.K;
  K.n = T->n;
  K.rowptr = T->rowptr;
  K.col = T->col;
  K.val = W.jval;
  K.perm = nullptr;
  K.dinv = W.dinv;
  K.rhs = W.F;
  K.rhs_scale = -1.0;
  K.x = W.delta;
  K.x_zero = 1;
  K.r = W.r;
  K.rhat = W.rhat;
  K.p = W.p;
  K.v = W.v;
  K.s = W.s;
  K.t = W.t;
  K.z = W.z;
  K.phat = W.phat;
  K.rh = W.rh;
  K.vh = W.vh;
  K.rtol = opts.krylov_rtol;
  K.max_iter = opts.max_krylov;
}

// Contiguous ranges of row blocks balanced by slots.
void split_blocks(const egfem_tensor_s* T, const std::vector<int32_t>& hblk, int g, std::vector<int32_t>& out) {
  const int64_t nb = T->row_blocks;
  const int64_t S = T->slots;
  out.assign(g + 1, 0);
  int64_t b = 0;
  for (int w = 1; w < g; ++w) {
    const int64_t target = S * w / g;
    while (b < nb && T->h_rowptr[hblk[b]] < target) ++b;
    // every member keeps at least one block
    b = std::max<int64_t>(b, out[w - 1] + 1);
    b = std::min<int64_t>(b, nb - (g - w));
    out[w] = (int32_t)b;
  }
  out[g] = (int32_t)nb;
}

}  // namespace

extern "C" {

int egfem_batch_create(int count, const egfem_tensor_t* Ts, const egfem_problem* ps, double* const* us,
                       const egfem_newton_opts* o, int threads, double weight_exp, egfem_batch_t* out) {
  using namespace egfem;
  if (!out) return fail(EGFEM_ERR_ARG, "out is null");
  *out = nullptr;
  if (count <= 0 || !Ts || !ps || !us) return fail(EGFEM_ERR_ARG, "null argument or count <= 0");
  if (threads != 0 && threads != 512 && threads != 1024) return fail(EGFEM_ERR_ARG, "threads must be 512 or 1024");
  if (weight_exp < 0.0 || weight_exp > 4.0) return fail(EGFEM_ERR_ARG, "weight_exp out of range");
  egfem_newton_opts opts;
  int rc0 = batch_opts(o, &opts);
  if (rc0 == EGFEM_OK) rc0 = batch_handles(count, Ts, us);
  if (rc0 != EGFEM_OK) return rc0;
  egfem_batch_s* B = new egfem_batch_s();
  B->count = count;
  B->NT = threads ? threads : 512;
  B->Ts.assign(Ts, Ts + count);
  // one row shape for the launch: the longest row over the instances
  int lanes = 4, max_row = 0;
  for (int m = 0; m < count; ++m) {
    lanes = std::max(lanes, Ts[m]->krylov_lanes);
    max_row = std::max(max_row, Ts[m]->max_row_slots);
  }
  const int L = row_shape_for(max_row, lanes);
  B->L = L;
  const int cap = B->NT == 1024 ? cap_T<1024>(L) : cap_T<512>(L);
  if (cap < count) {
    free_batch(B);
    return fail(EGFEM_ERR_SHAPE, "more instances than co-resident workgroups");
  }
  // team sizes: share of the resident workgroups ~ slots^weight_exp, at least 1,
  // at most one member per row block and 256 members
  const double ex = weight_exp > 0.0 ? weight_exp : 1.5;
  std::vector<double> w(count);
  double wsum = 0.0;
  for (int m = 0; m < count; ++m) wsum += (w[m] = std::pow((double)Ts[m]->slots, ex));
  std::vector<int> g(count);
  int total = 0;
  for (int m = 0; m < count; ++m) {
    const int lim = (int)std::min<int64_t>(Ts[m]->row_blocks, 256);
    g[m] = std::max(1, std::min(lim, (int)std::floor(cap * w[m] / wsum)));
    total += g[m];
  }
  while (total > cap) {   // shrink the largest teams
    int mx = 0;
    for (int m = 1; m < count; ++m) if (g[m] > g[mx]) mx = m;
    --g[mx];
    --total;
  }
  B->team = g;
  B->G = total;

  // per-instance workspaces and descriptors
  std::vector<Inst> hi(count);
  std::vector<int32_t> wg2inst, wgblk;
  std::vector<int> wgblk_off(count);
  int first = 0;
  for (int m = 0; m < count; ++m) {
    egfem_tensor_s* T = Ts[m];
    int rc = ensure_workspace(T);
    if (rc != EGFEM_OK) {
      free_batch(B);
      return rc;
    }
    std::vector<int32_t> hblk(T->row_blocks + 1);
    if (hipMemcpy(hblk.data(), T->blk_row, hblk.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      free_batch(B);
      return fail(EGFEM_ERR_HIP, "copy of row blocks failed");
    }
    std::vector<int32_t> part;
    split_blocks(T, hblk, g[m], part);
    wgblk_off[m] = (int)wgblk.size();
    wgblk.insert(wgblk.end(), part.begin(), part.end());
    for (int q = 0; q < g[m]; ++q) wg2inst.push_back(m);
    Inst& I = hi[m];
    fill_inst(I, T, ps[m], us[m], opts);
    I.team_first = first;
    I.team_size = g[m];
    first += g[m];
  }
  // batch buffers
  B->ctrl_words = (size_t)count * dev::kCtrlWords;
  size_t red_words = 0;
  std::vector<size_t> red_off(count);
  for (int m = 0; m < count; ++m) {
    red_off[m] = red_words;
    red_words += (size_t)kRedSlots * dev::kMaxRed * g[m];
  }
  bool ok = hipMalloc((void**)&B->d_insts, count * sizeof(Inst)) == hipSuccess &&
            hipMalloc((void**)&B->d_wg2inst, wg2inst.size() * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_wgblk, wgblk.size() * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_ctrl, B->ctrl_words * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_red, red_words * 8) == hipSuccess &&
            hipMalloc((void**)&B->d_stats, (size_t)count * kStatsWords * 8) == hipSuccess &&
            hipHostMalloc((void**)&B->h_stats, (size_t)count * kStatsWords * 8, 0) == hipSuccess;
  if (!ok) {
    free_batch(B);
    return fail(EGFEM_ERR_OOM, "batch buffers");
  }
  for (int m = 0; m < count; ++m) {
    hi[m].wgblk = B->d_wgblk + wgblk_off[m];
    hi[m].ctrl = B->d_ctrl + (size_t)m * dev::kCtrlWords;
    hi[m].red = B->d_red + red_off[m];
    hi[m].stats = B->d_stats + (size_t)m * kStatsWords;
  }
  ok = hipMemcpy(B->d_insts, hi.data(), count * sizeof(Inst), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(B->d_wg2inst, wg2inst.data(), wg2inst.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(B->d_wgblk, wgblk.data(), wgblk.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    free_batch(B);
    return fail(EGFEM_ERR_HIP, "upload of batch descriptors failed");
  }
  B->opts.tol = opts.tol;
  B->opts.max_newton = opts.max_newton;
  B->opts.max_krylov = opts.max_krylov;
  B->opts.krylov_rtol = opts.krylov_rtol;
  B->opts.forcing = opts.forcing;
  B->opts.eta_max = opts.eta_max;
  B->opts.max_backtracks = opts.max_backtracks;
  *out = B;
  return EGFEM_OK;
}

int egfem_batch_create_sched(int count, const egfem_tensor_t* Ts, const egfem_problem* ps, double* const* us,
                             const egfem_newton_opts* o, int threads, double dur_exp, egfem_batch_t* out) {
  using namespace egfem;
  if (!out) return fail(EGFEM_ERR_ARG, "out is null");
  *out = nullptr;
  if (count <= 0 || !Ts || !ps || !us) return fail(EGFEM_ERR_ARG, "null argument or count <= 0");
  if (threads != 0 && threads != 256 && threads != 512) return fail(EGFEM_ERR_ARG, "threads must be 256 or 512");
  if (!(dur_exp >= 0.0) || dur_exp > 4.0) return fail(EGFEM_ERR_ARG, "dur_exp out of range");
  egfem_newton_opts opts;
  int rc = batch_opts(o, &opts);
  if (rc == EGFEM_OK) rc = batch_handles(count, Ts, us);
  if (rc != EGFEM_OK) return rc;
  for (int m = 0; m < count; ++m) {
    if (Ts[m]->max_row_slots > kResidentRow)
      return fail(EGFEM_ERR_ARG, "rows of more than 8 entries: the resident teams do not apply");
    if (Ts[m]->n >= (int64_t(1) << 28)) return fail(EGFEM_ERR_SHAPE, "instance too large for the resident teams");
  }
  const int NT = threads ? threads : 256;
  const int cap = NT == 512 ? cap_sched<512>() : cap_sched<256>();
  if (cap < 1) return fail(EGFEM_ERR_HIP, "the scheduled batch kernel cannot be resident");
  egfem_batch_s* B = new egfem_batch_s();
  B->kind = 1;
  B->count = count;
  B->NT = NT;
  B->Ts.assign(Ts, Ts + count);
  // members: a compact partition of the rows into parts of at most NT rows
  // (the Krylov rows, one per thread) and, for the residual and the Jacobian,
  // consecutive row blocks balanced by slots
  std::vector<int> g(count);
  std::vector<int32_t> wgblk, kr, rlist, nbr;
  std::vector<int> wgblk_off(count), kr_off(count), nbr_off(count);
  std::vector<int64_t> rlist_off(count);
  std::vector<int16_t> kloc;
  std::vector<int64_t> kloc_off(count);
  for (int m = 0; m < count; ++m) {
    egfem_tensor_s* T = Ts[m];
    if ((rc = ensure_workspace(T)) != EGFEM_OK) {
      free_batch(B);
      return rc;
    }
    if (T->h_coords.empty()) {
      free_batch(B);
      return fail(EGFEM_ERR_ARG, "a handle without node coordinates cannot be partitioned");
    }
    std::vector<int32_t> hblk(T->row_blocks + 1);
    if (hipMemcpy(hblk.data(), T->blk_row, hblk.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      free_batch(B);
      return fail(EGFEM_ERR_HIP, "copy of row blocks failed");
    }
    int gm = (int)((T->n + NT - 1) / NT);
    CompactPartition cp;
    for (;;) {
      if (gm > cap || gm > kMaxKrylovBlocks || gm > T->row_blocks) {
        free_batch(B);
        return fail(EGFEM_ERR_SHAPE, "an instance needs more resident workgroups than the GPU holds");
      }
      if ((rc = make_compact_partition(T->dim, T->h_coords.data(), T->n, T->h_rowptr.data(), T->h_col.data(), gm,
                                       cp)) != EGFEM_OK) {
        free_batch(B);
        return rc;
      }
      if (cp.maxrows <= NT) break;
      ++gm;
    }
    g[m] = gm;
    std::vector<int32_t> part;
    split_blocks(T, hblk, gm, part);
    wgblk_off[m] = (int)wgblk.size();
    wgblk.insert(wgblk.end(), part.begin(), part.end());
    kr_off[m] = (int)kr.size();
    kr.insert(kr.end(), cp.kr.begin(), cp.kr.end());
    rlist_off[m] = (int64_t)rlist.size();
    rlist.insert(rlist.end(), cp.rlist.begin(), cp.rlist.end());
    nbr_off[m] = (int)nbr.size();
    nbr.insert(nbr.end(), cp.nbr.begin(), cp.nbr.end());
    kloc_off[m] = (int64_t)kloc.size();
    kloc.insert(kloc.end(), cp.kloc.begin(), cp.kloc.end());
  }
  // list scheduling: instances by estimated duration (n^dur_exp), longest
  // first, each on the window of g[m] consecutive workgroups that frees first
  const double ex = dur_exp > 0.0 ? dur_exp : 0.5;
  std::vector<double> dur(count);
  for (int m = 0; m < count; ++m) dur[m] = std::pow((double)Ts[m]->n, ex);
  std::vector<int> order(count);
  for (int m = 0; m < count; ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dur[a] > dur[b]; });
  std::vector<double> finish(cap, 0.0);
  std::vector<std::vector<int2>> lists(cap);
  int used = 0;
  for (int m : order) {
    int bp = 0;
    double bs = DBL_MAX;
    for (int p0 = 0; p0 + g[m] <= cap; ++p0) {
      double st0 = 0.0;
      for (int w = p0; w < p0 + g[m]; ++w) st0 = std::max(st0, finish[w]);
      if (st0 < bs) {
        bs = st0;
        bp = p0;
      }
    }
    for (int w = bp; w < bp + g[m]; ++w) {
      finish[w] = bs + dur[m];
      lists[w].push_back(make_int2(m, w - bp));
    }
    used = std::max(used, bp + g[m]);
  }
  B->makespan = *std::max_element(finish.begin(), finish.end());
  std::vector<int32_t> sptr(used + 1, 0);
  std::vector<int2> slist;
  for (int w = 0; w < used; ++w) {
    slist.insert(slist.end(), lists[w].begin(), lists[w].end());
    sptr[w + 1] = (int32_t)slist.size();
  }
  B->team = g;
  B->G = used;
  // buffers and descriptors
  B->ctrl_words = (size_t)count * dev::kCtrlWords;
  size_t red_words = 0;
  std::vector<size_t> red_off(count);
  for (int m = 0; m < count; ++m) {
    red_off[m] = red_words;
    red_words += (size_t)kRedSlots * dev::kMaxRed * g[m];
  }
  bool ok = hipMalloc((void**)&B->d_insts, count * sizeof(Inst)) == hipSuccess &&
            hipMalloc((void**)&B->d_wgblk, wgblk.size() * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_ctrl, B->ctrl_words * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_red, red_words * 8) == hipSuccess &&
            hipMalloc((void**)&B->d_stats, (size_t)count * kStatsWords * 8) == hipSuccess &&
            hipHostMalloc((void**)&B->h_stats, (size_t)count * kStatsWords * 8, 0) == hipSuccess &&
            hipMalloc((void**)&B->d_sched_ptr, sptr.size() * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_sched_list, std::max<size_t>(slist.size(), 1) * sizeof(int2)) == hipSuccess &&
            hipMalloc((void**)&B->d_kloc, std::max<size_t>(kloc.size(), 1) * 2) == hipSuccess &&
            hipMalloc((void**)&B->d_kr, kr.size() * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_rlist, std::max<size_t>(rlist.size(), 1) * 4) == hipSuccess &&
            hipMalloc((void**)&B->d_nbr, std::max<size_t>(nbr.size(), 1) * 4) == hipSuccess;
  if (!ok) {
    free_batch(B);
    return fail(EGFEM_ERR_OOM, "batch buffers");
  }
  std::vector<Inst> hi(count);
  for (int m = 0; m < count; ++m) {
    Inst& I = hi[m];
    fill_inst(I, Ts[m], ps[m], us[m], opts);
    I.K.kloc = B->d_kloc + kloc_off[m];
    I.K.rlist = B->d_rlist + rlist_off[m];
    I.K.cheb_steps = Ts[m]->krylov_precond;
    I.K.cheb_ratio = Ts[m]->krylov_cheb_ratio;
    I.kr = B->d_kr + kr_off[m];
    I.nbr = B->d_nbr + nbr_off[m];
    I.team_first = 0;
    I.team_size = g[m];
    I.wgblk = B->d_wgblk + wgblk_off[m];
    I.ctrl = B->d_ctrl + (size_t)m * dev::kCtrlWords;
    I.red = B->d_red + red_off[m];
    I.stats = B->d_stats + (size_t)m * kStatsWords;
  }
  ok = hipMemcpy(B->d_insts, hi.data(), count * sizeof(Inst), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(B->d_wgblk, wgblk.data(), wgblk.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(B->d_sched_ptr, sptr.data(), sptr.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       (slist.empty() ||
        hipMemcpy(B->d_sched_list, slist.data(), slist.size() * sizeof(int2), hipMemcpyHostToDevice) ==
            hipSuccess) &&
       (kloc.empty() || hipMemcpy(B->d_kloc, kloc.data(), kloc.size() * 2, hipMemcpyHostToDevice) == hipSuccess) &&
       hipMemcpy(B->d_kr, kr.data(), kr.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
       (rlist.empty() || hipMemcpy(B->d_rlist, rlist.data(), rlist.size() * 4, hipMemcpyHostToDevice) == hipSuccess) &&
       (nbr.empty() || hipMemcpy(B->d_nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
  if (!ok) {
    free_batch(B);
    return fail(EGFEM_ERR_HIP, "upload of batch descriptors failed");
  }
  B->opts.tol = opts.tol;
  B->opts.max_newton = opts.max_newton;
  B->opts.max_krylov = opts.max_krylov;
  B->opts.krylov_rtol = opts.krylov_rtol;
  B->opts.forcing = opts.forcing;
  B->opts.eta_max = opts.eta_max;
  B->opts.max_backtracks = opts.max_backtracks;
  *out = B;
  return EGFEM_OK;
}

// One run: zero the control words (fill kernel, graph-safe), the persistent
// launch, statistics to pinned host memory.
static int batch_enqueue(egfem_batch_t B, int zero_init, hipStream_t st) {
  using namespace egfem;
  EGFEM_HIP_CHECK(launch_fill_u32(B->d_ctrl, 0u, (int64_t)B->ctrl_words, st));
  BatchOpts O = B->opts;
  O.zero_init = zero_init ? 1 : 0;
  hipError_t e;
  if (B->kind == 1)
    e = B->NT == 512 ? launch_sched<512>(B->d_insts, B->d_sched_ptr, B->d_sched_list, O, (unsigned)B->G, st)
                     : launch_sched<256>(B->d_insts, B->d_sched_ptr, B->d_sched_list, O, (unsigned)B->G, st);
  else
    e = B->NT == 1024 ? launch_T<1024>(B->L, B->d_insts, B->d_wg2inst, O, (unsigned)B->G, st)
                      : launch_T<512>(B->L, B->d_insts, B->d_wg2inst, O, (unsigned)B->G, st);
  if (e != hipSuccess) return fail(EGFEM_ERR_HIP, std::string("batched launch failed: ") + hipGetErrorString(e));
  EGFEM_HIP_CHECK(hipMemcpyAsync(B->h_stats, B->d_stats, (size_t)B->count * kStatsWords * 8,
                                 hipMemcpyDeviceToHost, st));
  return EGFEM_OK;
}

int egfem_batch_run(egfem_batch_t B, int zero_init, void* stream) {
  if (!B) return egfem::fail(EGFEM_ERR_ARG, "null batch");
  return batch_enqueue(B, zero_init, (hipStream_t)stream);
}

int egfem_batch_graph_run(egfem_batch_t B, int zero_init, void* stream) {
  using namespace egfem;
  if (!B) return fail(EGFEM_ERR_ARG, "null batch");
  hipStream_t st = (hipStream_t)stream;
  if (!B->exec || B->graph_zero_init != (zero_init ? 1 : 0)) {
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    // capture on a plan-owned stream (the caller's may be the legacy null
    // stream, which cannot be captured); the graph is launched on `stream`
    if (!B->cap_stream) EGFEM_HIP_CHECK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
    EGFEM_HIP_CHECK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue(B, zero_init, B->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (rc != EGFEM_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(EGFEM_ERR_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    B->graph = g;
    EGFEM_HIP_CHECK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
    B->graph_zero_init = zero_init ? 1 : 0;
  }
  EGFEM_HIP_CHECK(hipGraphLaunch(B->exec, st));
  return EGFEM_OK;
}

int egfem_batch_stats(egfem_batch_t B, egfem_newton_stats* stats, void* stream) {
  using namespace egfem;
  if (!B) return fail(EGFEM_ERR_ARG, "null batch");
  EGFEM_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  int worst = EGFEM_OK;
  for (int m = 0; m < B->count; ++m) {
    const double* s = B->h_stats + (size_t)m * kStatsWords;
    const int status = (int)s[0];
    if (status == EGFEM_ERR_HIP) return fail(EGFEM_ERR_HIP, "batched Newton: a team barrier timed out");
    worst = std::max(worst, status);
    if (!stats) continue;
    egfem_newton_stats& o = stats[m];
    std::memset(&o, 0, sizeof(o));
    o.status = status;
    o.newton_iters = (int)s[1];
    o.krylov_iters = (int)s[2];
    o.backtracks = (int)s[3];
    o.res0 = s[4];
    o.res = s[5];
    // the streaming teams' BiCGStab streams its rows; the scheduled teams run
    // the register-resident form (block-Jacobi unless the handle asks Jacobi)
    if (o.newton_iters > 0)
      o.krylov_kernels = B->kind == 1 ? (1 | (B->Ts[m]->krylov_precond > 0 ? 4 : 0)) : 2;
    for (int k = 0; k < EGFEM_HIST && k < o.newton_iters; ++k) {
      o.res_hist[k] = s[6 + k];
      o.krylov_hist[k] = (int)s[6 + EGFEM_HIST + k];
    }
    // the Krylov solve of a step that was not accepted is reported too
    for (int k = 0; k < EGFEM_HIST && k <= o.newton_iters; ++k) {
      o.krylov_status_hist[k] = (int)s[6 + 2 * EGFEM_HIST + k];
      o.krylov_relres_hist[k] = s[6 + 3 * EGFEM_HIST + k];
    }
  }
  return worst;
}

int egfem_batch_teams(egfem_batch_t B, int* team_sizes, int* total_workgroups) {
  if (!B) return egfem::fail(EGFEM_ERR_ARG, "null batch");
  if (team_sizes)
    for (int m = 0; m < B->count; ++m) team_sizes[m] = B->team[m];
  if (total_workgroups) *total_workgroups = B->G;
  return EGFEM_OK;
}

void egfem_batch_destroy(egfem_batch_t B) { free_batch(B); }

int egfem_batch_autotune(int count, const egfem_tensor_t* Ts, const egfem_problem* ps, double* const* us,
                         const egfem_newton_opts* o, int* best_kind, int* best_threads, double* best_exp,
                         double* best_ms, void* stream) {
  using namespace egfem;
  if (count < 1) return fail(EGFEM_ERR_ARG, "count must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  std::vector<egfem_newton_stats> stats((size_t)count);
  // the scheduled resident teams apply to P1 handles with rows of <= 8 entries
  bool sched_ok = true;
  for (int m = 0; m < count; ++m)
    if (!Ts || !Ts[m] || Ts[m]->w2 || Ts[m]->max_row_slots > kResidentRow) sched_ok = false;
  struct Cand {
    int kind, threads;
    double ex;
  };
  std::vector<Cand> cands;
  for (int threads : {512, 1024})
    for (double wexp : {1.0, 1.5, 2.0}) cands.push_back({0, threads, wexp});
  if (sched_ok)
    for (int threads : {256, 512})
      for (double dexp : {0.5, 1.0}) cands.push_back({1, threads, dexp});
  double bt = DBL_MAX;
  Cand best{-1, 0, 0.0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EGFEM_HIP_CHECK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(EGFEM_ERR_HIP, "hipEventCreate failed");
  }
  int rc = EGFEM_OK;
  for (const Cand& c : cands) {
    egfem_batch_t B = nullptr;
    rc = c.kind == 1 ? egfem_batch_create_sched(count, Ts, ps, us, o, c.threads, c.ex, &B)
                     : egfem_batch_create(count, Ts, ps, us, o, c.threads, c.ex, &B);
    if (rc == EGFEM_ERR_SHAPE) {   // this shape does not fit the resident workgroups
      rc = EGFEM_OK;
      continue;
    }
    if (rc != EGFEM_OK) break;
    // a first run warms the handles and the plan; the second is timed
    bool good = true;
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && rc == EGFEM_OK; ++rep) {
      if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(EGFEM_ERR_HIP, "hipEventRecord failed");
      if (rc == EGFEM_OK) rc = egfem_batch_run(B, 1, st);
      if (rc == EGFEM_OK && rep == 1 && hipEventRecord(e1, st) != hipSuccess)
        rc = fail(EGFEM_ERR_HIP, "hipEventRecord failed");
      if (rc == EGFEM_OK) {
        const int worst = egfem_batch_stats(B, stats.data(), st);
        if (worst < 0) rc = worst;
      }
    }
    // every instance converged, or stopped at the rounding floor of ||F||
    for (int m = 0; rc == EGFEM_OK && m < count; ++m)
      good = good && (stats[m].status == EGFEM_OK || stats[m].status == EGFEM_STAGNATED);
    if (rc == EGFEM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = fail(EGFEM_ERR_HIP, "hipEventElapsedTime failed");
    egfem_batch_destroy(B);
    if (rc != EGFEM_OK) break;
    if (good && ms < bt) {
      bt = ms;
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != EGFEM_OK) return rc;
  if (best.kind < 0) return fail(EGFEM_ERR_ARG, "no batch shape converged");
  if (best_kind) *best_kind = best.kind;
  if (best_threads) *best_threads = best.threads;
  if (best_exp) *best_exp = best.ex;
  if (best_ms) *best_ms = bt;
  return EGFEM_OK;
}

int egfem_newton_batched(int count, const egfem_tensor_t* Ts, const egfem_problem* ps, double* const* us,
                         const egfem_newton_opts* o, egfem_newton_stats* stats, void* stream) {
  egfem_batch_t B = nullptr;
  int rc = egfem_batch_create(count, Ts, ps, us, o, o ? o->krylov_threads : 0, 0.0, &B);
  if (rc != EGFEM_OK) return rc;
  rc = egfem_batch_run(B, 0, stream);
  if (rc == EGFEM_OK) rc = egfem_batch_stats(B, stats, stream);
  egfem_batch_destroy(B);
  return rc;
}

}  // extern "C"
