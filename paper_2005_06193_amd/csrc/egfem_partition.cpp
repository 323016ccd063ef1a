// Compact row partition of the register-resident Krylov solvers: recursive
// coordinate bisection of the nodes into G parts of balanced size (one part
// per workgroup), so that each workgroup's rows form a compact patch of the
// mesh and its diagonal block of J holds most of the rows' couplings (the
// block-Jacobi preconditioner works on that block).
#include <algorithm>
#include <numeric>

#include "egfem_internal.h"

namespace egfem {

namespace {

// Split idx[lo, hi) into `parts` parts along the axis of largest extent,
// recursively; part q receives idx[kr[first + q], kr[first + q + 1]).
void rcb(const double* X, int dim, std::vector<int32_t>& idx, size_t lo, size_t hi, int parts, int first,
         std::vector<int32_t>& kr) {
  if (parts == 1) {
    kr[first + 1] = (int32_t)hi;
    return;
  }
  double mn[3] = {0.0, 0.0, 0.0}, mx[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < dim; ++r) {
    mn[r] = 1e300;
    mx[r] = -1e300;
  }
  for (size_t q = lo; q < hi; ++q)
    for (int r = 0; r < dim; ++r) {
      const double v = X[(size_t)idx[q] * dim + r];
      mn[r] = std::min(mn[r], v);
      mx[r] = std::max(mx[r], v);
    }
  int ax = 0;
  for (int r = 1; r < dim; ++r)
    if (mx[r] - mn[r] > mx[ax] - mn[ax]) ax = r;
  // total order (coordinate, node id): the partition is deterministic
  std::sort(idx.begin() + lo, idx.begin() + hi, [&](int32_t a, int32_t b) {
    const double va = X[(size_t)a * dim + ax], vb = X[(size_t)b * dim + ax];
    return va < vb || (va == vb && a < b);
  });
  const int h = parts / 2;
  const size_t cut = lo + (hi - lo) * (size_t)h / (size_t)parts;
  rcb(X, dim, idx, lo, cut, h, first, kr);
  rcb(X, dim, idx, cut, hi, parts - h, first + h, kr);
}

}  // namespace

void uniform_neighbor_lists(std::vector<int32_t>& nbr, int G) {
  // the point-to-point synchronisation and the team barrier do not mix: one
  // overflowing list sends every workgroup to the team barrier
  bool overflow = false;
  for (int g = 0; g < G; ++g) overflow = overflow || nbr[(size_t)g * (kMaxNbrLists + 1)] < 0;
  if (overflow)
    for (int g = 0; g < G; ++g) nbr[(size_t)g * (kMaxNbrLists + 1)] = -1;
}

int make_compact_partition(int dim, const double* X, int64_t n, const int32_t* rowptr, const int32_t* col, int G,
                           CompactPartition& out, const uint8_t* skip) {
  if (n <= 0 || G < 1 || dim < 1 || dim > 3) return fail(EGFEM_ERR_ARG, "invalid partition request");
  // the rows to partition: all, or those not marked in skip
  std::vector<int32_t> idx;
  idx.reserve((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    if (!skip || !skip[i]) idx.push_back((int32_t)i);
  const int64_t nr = (int64_t)idx.size();
  if (nr == 0 || G > nr) return fail(EGFEM_ERR_ARG, "invalid partition request");
  out.kr.assign(G + 1, 0);
  rcb(X, dim, idx, 0, (size_t)nr, G, 0, out.kr);
  std::vector<int32_t> owner(n, -1), pos(n, 0);
  out.maxrows = 0;
  for (int g = 0; g < G; ++g) {
    // rows of a part in ascending order
    std::sort(idx.begin() + out.kr[g], idx.begin() + out.kr[g + 1]);
    out.maxrows = std::max(out.maxrows, out.kr[g + 1] - out.kr[g]);
    for (int32_t q = out.kr[g]; q < out.kr[g + 1]; ++q) {
      owner[idx[q]] = g;
      pos[idx[q]] = q - out.kr[g];
    }
  }
  if (out.maxrows > 32767) return fail(EGFEM_ERR_SHAPE, "partition parts too large");
  out.rlist = idx;
  // per slot: the row-local position of its column when the same part owns it, else -1
  // (rows left out own no part and keep -1)
  out.kloc.assign((size_t)rowptr[n], -1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s)
      if (owner[i] >= 0 && owner[col[s]] == owner[i]) out.kloc[s] = (int16_t)pos[col[s]];
  // neighbour lists: the other parts owning a column of this part's rows
  out.nbr.assign((size_t)G * (kMaxNbrLists + 1), 0);
  for (int g = 0; g < G; ++g) {
    int32_t* lst = out.nbr.data() + (size_t)g * (kMaxNbrLists + 1);
    int cnt = 0;
    for (int32_t q = out.kr[g]; q < out.kr[g + 1] && cnt >= 0; ++q) {
      const int32_t i = idx[q];
      for (int32_t s = rowptr[i]; s < rowptr[i + 1] && cnt >= 0; ++s) {
        const int o = owner[col[s]];
        if (o == g || o < 0) continue;   // own part, or a row left out (never published)
        bool seen = false;
        for (int m = 0; m < cnt; ++m) seen = seen || lst[1 + m] == o;
        if (seen) continue;
        if (cnt == kMaxNbrLists) cnt = -1;   // too many: the team barrier
        else lst[1 + cnt++] = o;
      }
    }
    lst[0] = cnt;
  }
  uniform_neighbor_lists(out.nbr, G);
  return EGFEM_OK;
}

}  // namespace egfem
