// Offline phase: assemble the EGFEM tensor, the stiffness and the mass matrix
// of a P1 simplex mesh and lay them out as slot-aligned fiber streams.
//
// Tensor (eq. egfem_terms with W_h = V_h = P1):
//   stiffness form  T_ijk = sum_e int_e phi_k grad phi_j . grad phi_i
//                         = sum_e K^e_ij / (d+1)       (grad phi constant, int_e phi_k = |e|/(d+1))
//   mass form       T_ijk = sum_e int_e phi_i phi_j phi_k
//                         = sum_e d! |e| alpha! / (d+3)!  (exact simplex monomial integral)
//   convection form T_ijk = sum_e int_e phi_k phi_j sum_d d_d phi_i   (tensor N of Sec. 5.2)
//                         = sum_e (sum_d d_d lambda_i) M^e_jk      (gradient constant per cell)
// K_ij = sum_e |e| grad phi_j . grad phi_i,  M_ij = sum_e |e| (1 + delta_ij) / ((d+1)(d+2)).
//
// W_h = I_k (Case 3 of Sec. 3.1): k = e * Q + q runs over the points of a fixed
// quadrature rule in every cell, eta_k is the functional f -> w_q |e| f(x_q):
//   stiffness T_ijk = w_q |e| grad phi_j . grad phi_i,  mass T_ijk = w_q |e| phi_j(x_q) phi_i(x_q);
// the rule is 2-point Gauss in 1D and the degree-2 interior rules with 3 (2D)
// and 4 (3D) points.
//
// W_h = P2 (Case 1 of Sec. 3.1; egfem_build_tensor_w): k runs over the P2 dofs
// (vertices 0..N-1, then the edges in ascending (min, max) vertex order) with
// eta_k the P2 nodal basis: vertex lambda(2 lambda - 1), edge 4 lambda_x lambda_y;
// every P2 dof coupled to row i is a vertex or an edge of a cell of i, so both
// of its endpoints are columns of row i.
//
// Layout (all indices int32, values float64):
//   CSR pattern of the P1 adjacency including the diagonal: rowptr, col.
//   A-stream: for slot s = (i,j) the fiber kptrA[s]..kptrA[s+1] of (k, T_ijk), k ascending.
//   B-stream: for slot s = (i,k) the fiber jptrB[s]..jptrB[s+1] of (j, T_ijk), j ascending.
//   For tensors with T_ijk = T_ikj (mass, convection) B == A and is not stored twice.
//   tperm[s] = slot of (j,i); diag[i] = slot of (i,i).
//   Row blocks: runs of rows that fit the LDS capacities of the tensor kernels.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "egfem_internal.h"

namespace {

struct Geom {
  double vol;          // |e|
  double G[4][3];      // grad lambda_a
};

bool cell_geometry(int dim, const double* X, const int32_t* c, Geom& g) {
  double B[3][3] = {{0}};   // B[r][m] = x_{m+1}[r] - x_0[r]
  for (int m = 0; m < dim; ++m)
    for (int r = 0; r < dim; ++r) B[r][m] = X[(int64_t)c[m + 1] * dim + r] - X[(int64_t)c[0] * dim + r];
  double inv[3][3] = {{0}};
  double det;
  if (dim == 1) {
    det = B[0][0];
    inv[0][0] = 1.0 / det;
  } else if (dim == 2) {
    det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    inv[0][0] = B[1][1] / det;
    inv[0][1] = -B[0][1] / det;
    inv[1][0] = -B[1][0] / det;
    inv[1][1] = B[0][0] / det;
  } else {
    const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
    const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
    const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
    det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
    inv[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
    inv[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
    inv[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
    inv[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
    inv[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
  }
  if (!(det != 0.0) || !std::isfinite(det)) return false;
  double fact = 1.0;
  for (int m = 2; m <= dim; ++m) fact *= m;
  g.vol = std::fabs(det) / fact;
  // lambda_m(x) = (B^{-1}(x - x0))_{m-1} for m >= 1, lambda_0 = 1 - sum
  for (int r = 0; r < dim; ++r) {
    double s = 0.0;
    for (int m = 0; m < dim; ++m) {
      g.G[m + 1][r] = inv[m][r];
      s += inv[m][r];
    }
    g.G[0][r] = -s;
  }
  return true;
}

// Every array gets kPad zero elements past its end: the row-block stages load
// at indices clamped to a range's last element, which for an empty range is
// the element just past it.
constexpr size_t kPad = 16;

template <typename T>
int upload(const std::vector<T>& h, T** d, int64_t* bytes) {
  const size_t nb = (h.size() + kPad) * sizeof(T);
  hipError_t e = hipMalloc((void**)d, nb);
  if (e != hipSuccess) return egfem::fail(EGFEM_ERR_OOM, "hipMalloc of tensor stream failed");
  *bytes += (int64_t)nb;
  e = hipMemset(*d, 0, nb);
  if (e == hipSuccess && !h.empty())
    e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return egfem::fail(EGFEM_ERR_HIP, "upload of tensor stream failed");
  return EGFEM_OK;
}


// d! prod alpha_m! / (d + |alpha|)!: int_e prod lambda_m^alpha_m / |e|
double mono(int dim, const int* alpha) {
  int tot = 0;
  double num = 1.0;
  for (int m = 0; m <= dim; ++m) {
    tot += alpha[m];
    for (int f = 2; f <= alpha[m]; ++f) num *= f;
  }
  for (int f = 2; f <= dim; ++f) num *= f;
  double den = 1.0;
  for (int f = 2; f <= dim + tot; ++f) den *= f;
  return num / den;
}

// int_e m eta_c / |e| for the local P2 dof c (c < nl: vertex c; else the
// local edge ledge[c - nl]), where m is the barycentric monomial with
// exponents base[].
double p2_int_base(int dim, const int base[4], int c, const int (*ledge)[2]) {
  const int nl = dim + 1;
  if (c < nl) {
    int x1[4], x2[4];
    for (int m = 0; m < 4; ++m) x1[m] = x2[m] = base[m];
    x1[c] += 2;
    x2[c] += 1;
    return 2.0 * mono(dim, x1) - mono(dim, x2);
  }
  int x[4];
  for (int m = 0; m < 4; ++m) x[m] = base[m];
  x[ledge[c - nl][0]]++;
  x[ledge[c - nl][1]]++;
  return 4.0 * mono(dim, x);
}

// int_e eta_c / |e| and int_e lambda_a lambda_b eta_c / |e| (with_ab).
double p2_int(int dim, int a, int b, int c, const int (*ledge)[2], bool with_ab) {
  int base[4] = {0, 0, 0, 0};
  if (with_ab) {
    base[a]++;
    base[b]++;
  }
  return p2_int_base(dim, base, c, ledge);
}

// int_e lambda_b eta_c / |e| (convection form).
double p2_int1(int dim, int b, int c, const int (*ledge)[2]) {
  int base[4] = {0, 0, 0, 0};
  base[b]++;
  return p2_int_base(dim, base, c, ledge);
}

int build_impl(int dim, int64_t n_nodes, const double* coords, int64_t n_cells, const int32_t* cells, int form,
               int wspace, double drop_rel, egfem_tensor_t* out) {
  using namespace egfem;
  if (!out) return fail(EGFEM_ERR_ARG, "out is null");
  *out = nullptr;
  if (dim < 1 || dim > 3) return fail(EGFEM_ERR_ARG, "dim must be 1, 2 or 3");
  if (form != EGFEM_FORM_STIFF && form != EGFEM_FORM_MASS && form != EGFEM_FORM_CONV)
    return fail(EGFEM_ERR_ARG, "unknown form");
  if (wspace != EGFEM_W_P1 && wspace != EGFEM_W_P2 && wspace != EGFEM_W_IQ && wspace != EGFEM_W_P0)
    return fail(EGFEM_ERR_ARG, "unknown W space");
  if (wspace == EGFEM_W_P0 && form == EGFEM_FORM_CONV)
    return fail(EGFEM_ERR_ARG, "the convection form is built with W_h = P1, P2 or I_k only");
  const bool w2 = (wspace != EGFEM_W_P1);     // a coefficient space with W-slots
  const bool wq = (wspace == EGFEM_W_IQ);
  const bool wcell = (wspace == EGFEM_W_P0);   // one coefficient per cell
  // quadrature rule of W_h = I_k: barycentrics (padded to 4) and weights / |e|
  int nq = 0;
  double qlam[4][4] = {{0}}, qw[4] = {0};
  if (wcell) {
    // the indicator of the cell: one "point" with weight 1 (|e| folded into the
    // values); no barycentric weights are used
    nq = 1;
    qw[0] = 1.0;
  } else if (wq) {
    if (dim == 1) {
      nq = 2;
      const double x0 = 0.5 - 0.5 / std::sqrt(3.0), x1 = 0.5 + 0.5 / std::sqrt(3.0);
      qlam[0][0] = 1.0 - x0;
      qlam[0][1] = x0;
      qlam[1][0] = 1.0 - x1;
      qlam[1][1] = x1;
      qw[0] = qw[1] = 0.5;
    } else if (dim == 2) {
      nq = 3;
      for (int q = 0; q < 3; ++q) {
        for (int m = 0; m < 3; ++m) qlam[q][m] = (q == m) ? 2.0 / 3.0 : 1.0 / 6.0;
        qw[q] = 1.0 / 3.0;
      }
    } else {
      nq = 4;
      const double qa = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0, qb = (5.0 - std::sqrt(5.0)) / 20.0;
      for (int q = 0; q < 4; ++q) {
        for (int m = 0; m < 4; ++m) qlam[q][m] = (q == m) ? qa : qb;
        qw[q] = 0.25;
      }
    }
  }
  if (!coords || !cells) return fail(EGFEM_ERR_ARG, "coords/cells null");
  if (n_nodes <= 0 || n_cells <= 0) return fail(EGFEM_ERR_SHAPE, "empty mesh");
  if (n_nodes >= (int64_t(1) << 31) || n_cells >= (int64_t(1) << 31))
    return fail(EGFEM_ERR_SHAPE, "mesh too large for int32 indices");
  if (!(drop_rel >= 0.0)) return fail(EGFEM_ERR_ARG, "drop_rel must be >= 0");
  const int nl = dim + 1;
  const int64_t N = n_nodes;

  // --- element geometry --------------------------------------------------
  std::vector<Geom> geo((size_t)n_cells);
  for (int64_t e = 0; e < n_cells; ++e) {
    const int32_t* c = cells + e * nl;
    for (int a = 0; a < nl; ++a)
      if (c[a] < 0 || c[a] >= N) return fail(EGFEM_ERR_MESH, "cell index out of range");
    for (int a = 0; a < nl; ++a)
      for (int b = a + 1; b < nl; ++b)
        if (c[a] == c[b]) return fail(EGFEM_ERR_MESH, "repeated vertex in a cell");
    if (!cell_geometry(dim, coords, c, geo[e])) return fail(EGFEM_ERR_MESH, "degenerate cell");
  }

  // --- node -> cell incidence -------------------------------------------
  std::vector<int64_t> nptr(N + 1, 0);
  for (int64_t e = 0; e < n_cells; ++e)
    for (int a = 0; a < nl; ++a) nptr[cells[e * nl + a] + 1]++;
  for (int64_t i = 0; i < N; ++i) {
    if (nptr[i + 1] == 0) return fail(EGFEM_ERR_MESH, "node not referenced by any cell");
    nptr[i + 1] += nptr[i];
  }
  std::vector<int32_t> ncell(nptr[N]);
  {
    std::vector<int64_t> fillp(nptr.begin(), nptr.end() - 1);
    for (int64_t e = 0; e < n_cells; ++e)
      for (int a = 0; a < nl; ++a) ncell[fillp[cells[e * nl + a]]++] = (int32_t)e;   // ascending e
  }

  // local integrals of the mass tensor: d! alpha! / (d+3)! by multiplicity pattern
  double fact_d = 1.0, fact_d3 = 1.0;
  for (int m = 2; m <= dim; ++m) fact_d *= m;
  for (int m = 2; m <= dim + 3; ++m) fact_d3 *= m;
  const double m3_aaa = fact_d * 6.0 / fact_d3;
  const double m3_aab = fact_d * 2.0 / fact_d3;
  const double m3_abc = fact_d * 1.0 / fact_d3;
  const double m2_diag = 2.0 / ((dim + 1.0) * (dim + 2.0));
  const double m2_off = 1.0 / ((dim + 1.0) * (dim + 2.0));

  // --- row pass: pattern, matrices and both fiber streams -----------------
  std::vector<int32_t> rowptr(N + 1, 0), col;
  std::vector<int32_t> kptrA(1, 0), kA, jptrB(1, 0), jB;
  std::vector<uint16_t> kRel, jRel;   // position of k (of j) among the row's columns
  std::vector<double> vA, vB, kval, mval;
  int64_t structural = 0;
  int max_row_slots = 0;
  std::vector<int32_t> cols;
  std::vector<double> acc;
  std::vector<unsigned char> present;
  std::vector<double> kacc, macc;
  // B == A exactly when T_ijk = T_ikj (never with W_h = P2: k and j live in
  // different spaces)
  const bool sym = (form != EGFEM_FORM_STIFF) && !w2;
  // W_h = P2: global edges (ascending (min, max)), per-row W-slot records
  const int ne_loc = nl * (nl - 1) / 2;
  int ledge[6][2];
  {
    int t = 0;
    for (int x = 0; x < nl; ++x)
      for (int y = x + 1; y < nl; ++y) {
        ledge[t][0] = x;
        ledge[t][1] = y;
        ++t;
      }
  }
  if ((wq || wcell) && n_cells * nq >= (int64_t(1) << 31)) return fail(EGFEM_ERR_SHAPE, "too many quadrature points");
  std::vector<int64_t> ekeys;   // min * N + max of every edge
  if (w2 && !wq) {
    ekeys.reserve((size_t)n_cells * ne_loc);
    for (int64_t e = 0; e < n_cells; ++e) {
      const int32_t* c = cells + e * nl;
      for (int t = 0; t < ne_loc; ++t) {
        const int64_t x = c[ledge[t][0]], y = c[ledge[t][1]];
        ekeys.push_back(std::min(x, y) * N + std::max(x, y));
      }
    }
    std::sort(ekeys.begin(), ekeys.end());
    ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
    if (N + (int64_t)ekeys.size() >= (int64_t(1) << 31)) return fail(EGFEM_ERR_SHAPE, "too many P2 dofs");
  }
  auto edge_id = [&](int64_t x, int64_t y) {
    const int64_t key = std::min(x, y) * N + std::max(x, y);
    return (int64_t)(std::lower_bound(ekeys.begin(), ekeys.end(), key) - ekeys.begin());
  };
  std::vector<int32_t> wrowptr(w2 ? N + 1 : 0, 0), wcol;
  std::vector<uint16_t> wpl, wql;   // row-local slot positions of a W-slot's endpoints
  std::vector<uint16_t> wpl2, wql2; // I_k: slots of the third and fourth vertex
  // symmetric half stream (T_ijk = T_ikj, W_h = P1): per slot (i, j) the
  // entries with k at or after j, the diagonal one halved
  std::vector<int32_t> kptrH(1, 0);
  std::vector<uint16_t> hRel;
  std::vector<double> vH;
  std::vector<uint8_t> wqi;         // I_k: point index of a W-slot
  std::vector<int64_t> redges;
  int max_row_wslots = 0;
  col.reserve((size_t)N * (dim == 3 ? 15 : 7));

  for (int64_t i = 0; i < N; ++i) {
    cols.clear();
    for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) {
      const int32_t* c = cells + (int64_t)ncell[q] * nl;
      for (int a = 0; a < nl; ++a) cols.push_back(c[a]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    const int nc = (int)cols.size();
    max_row_slots = std::max(max_row_slots, nc);
    auto lidx = [&](int32_t node) {
      return (int)(std::lower_bound(cols.begin(), cols.end(), node) - cols.begin());
    };
    if (wq || wcell) {
      // W-slots of row i: the points of its cells (ascending cell, then point);
      // for W_h = P0 the cells themselves
      const int ncl = (int)(nptr[i + 1] - nptr[i]);
      const int nw = ncl * nq;
      max_row_wslots = std::max(max_row_wslots, nw);
      acc.assign((size_t)nc * nw, 0.0);
      present.assign((size_t)nc * nw, 0);
      kacc.assign(nc, 0.0);
      macc.assign(nc, 0.0);
      for (int ce = 0; ce < ncl; ++ce) {
        const int64_t e = ncell[nptr[i] + ce];
        const int32_t* c = cells + e * nl;
        const Geom& g = geo[e];
        int a = 0;
        while (c[a] != (int32_t)i) ++a;
        int loc[4];
        for (int b = 0; b < nl; ++b) loc[b] = lidx(c[b]);
        // sum_d d_d lambda_a (convection form), rounding noise of a zero sum removed
        double gsum = 0.0, gabs = 0.0;
        for (int r = 0; r < dim; ++r) {
          gsum += g.G[a][r];
          gabs += std::fabs(g.G[a][r]);
        }
        if (std::fabs(gsum) <= 1e-12 * gabs) gsum = 0.0;
        for (int b = 0; b < nl; ++b) {
          double gg = 0.0;
          for (int r = 0; r < dim; ++r) gg += g.G[a][r] * g.G[b][r];
          const double kab = g.vol * gg;
          kacc[loc[b]] += kab;
          macc[loc[b]] += g.vol * (a == b ? m2_diag : m2_off);
          for (int q = 0; q < nq; ++q) {
            double val;
            if (wcell) val = (form == EGFEM_FORM_STIFF) ? kab : g.vol * (a == b ? m2_diag : m2_off);
            else if (form == EGFEM_FORM_STIFF) val = qw[q] * kab;
            else if (form == EGFEM_FORM_MASS) val = qw[q] * g.vol * qlam[q][a] * qlam[q][b];
            else val = qw[q] * g.vol * gsum * qlam[q][b];   // w_q |e| phi_b(x_q) sum_d d_d phi_a
            const size_t idx = (size_t)loc[b] * nw + (size_t)ce * nq + q;
            acc[idx] += val;
            present[idx] = 1;
          }
        }
      }
      double rowmax = 0.0;
      for (size_t t = 0; t < acc.size(); ++t)
        if (present[t]) {
          ++structural;
          rowmax = std::max(rowmax, std::fabs(acc[t]));
        }
      const double thr = drop_rel * rowmax;
      auto kept = [&](size_t t) { return present[t] && acc[t] != 0.0 && std::fabs(acc[t]) > thr; };
      auto wdof = [&](int kc) { return (int32_t)((int64_t)ncell[nptr[i] + kc / nq] * nq + kc % nq); };
      for (int jb = 0; jb < nc; ++jb) {
        col.push_back(cols[jb]);
        kval.push_back(kacc[jb]);
        mval.push_back(macc[jb]);
        for (int kc = 0; kc < nw; ++kc) {
          const size_t t = (size_t)jb * nw + kc;
          if (kept(t)) {
            kA.push_back(wdof(kc));
            kRel.push_back((uint16_t)kc);
            vA.push_back(acc[t]);
          }
        }
        kptrA.push_back((int32_t)kA.size());
      }
      for (int kc = 0; kc < nw; ++kc) {
        const int32_t* c = cells + (int64_t)ncell[nptr[i] + kc / nq] * nl;
        int sl[4];
        for (int m = 0; m < 4; ++m) sl[m] = lidx(c[m < nl ? m : 0]);
        wcol.push_back(wdof(kc));
        wpl.push_back((uint16_t)sl[0]);
        wql.push_back((uint16_t)sl[1]);
        wpl2.push_back((uint16_t)sl[2]);
        wql2.push_back((uint16_t)sl[3]);
        wqi.push_back((uint8_t)(kc % nq));
        for (int jb = 0; jb < nc; ++jb) {
          const size_t t = (size_t)jb * nw + kc;
          if (kept(t)) {
            jB.push_back(cols[jb]);
            jRel.push_back((uint16_t)jb);
            vB.push_back(acc[t]);
          }
        }
        jptrB.push_back((int32_t)jB.size());
      }
      if (col.size() >= (size_t)INT32_MAX || kA.size() >= (size_t)INT32_MAX || jB.size() >= (size_t)INT32_MAX ||
          wcol.size() >= (size_t)INT32_MAX)
        return fail(EGFEM_ERR_SHAPE, "more than 2^31 slots or tensor entries");
      wrowptr[i + 1] = (int32_t)wcol.size();
      rowptr[i + 1] = (int32_t)col.size();
      continue;
    }
    if (w2) {
      // W-slots of row i: its vertex dofs (the row's columns, same order),
      // then the edge dofs of its cells in ascending id
      redges.clear();
      for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) {
        const int32_t* c = cells + (int64_t)ncell[q] * nl;
        for (int t = 0; t < ne_loc; ++t) redges.push_back(edge_id(c[ledge[t][0]], c[ledge[t][1]]));
      }
      std::sort(redges.begin(), redges.end());
      redges.erase(std::unique(redges.begin(), redges.end()), redges.end());
      const int nw = nc + (int)redges.size();
      max_row_wslots = std::max(max_row_wslots, nw);
      acc.assign((size_t)nc * nw, 0.0);
      present.assign((size_t)nc * nw, 0);
      kacc.assign(nc, 0.0);
      macc.assign(nc, 0.0);
      for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) {
        const int64_t e = ncell[q];
        const int32_t* c = cells + e * nl;
        const Geom& g = geo[e];
        int a = 0;
        while (c[a] != (int32_t)i) ++a;
        int loc[4], wl[10];
        for (int b = 0; b < nl; ++b) loc[b] = wl[b] = lidx(c[b]);
        for (int t = 0; t < ne_loc; ++t) {
          const int64_t eid = edge_id(c[ledge[t][0]], c[ledge[t][1]]);
          wl[nl + t] = nc + (int)(std::lower_bound(redges.begin(), redges.end(), eid) - redges.begin());
        }
        // sum_d d_d lambda_a (convection form), rounding noise of a zero sum removed
        double gsum = 0.0, gabs = 0.0;
        for (int r = 0; r < dim; ++r) {
          gsum += g.G[a][r];
          gabs += std::fabs(g.G[a][r]);
        }
        if (std::fabs(gsum) <= 1e-12 * gabs) gsum = 0.0;
        for (int b = 0; b < nl; ++b) {
          double gg = 0.0;
          for (int r = 0; r < dim; ++r) gg += g.G[a][r] * g.G[b][r];
          const double kab = g.vol * gg;
          kacc[loc[b]] += kab;
          macc[loc[b]] += g.vol * (a == b ? m2_diag : m2_off);
          for (int cd = 0; cd < nl + ne_loc; ++cd) {
            double val;
            if (form == EGFEM_FORM_STIFF) val = kab * p2_int(dim, a, b, cd, ledge, false);
            else if (form == EGFEM_FORM_MASS) val = g.vol * p2_int(dim, a, b, cd, ledge, true);
            else val = gsum * g.vol * p2_int1(dim, b, cd, ledge);
            const size_t idx = (size_t)loc[b] * nw + wl[cd];
            acc[idx] += val;
            present[idx] = 1;
          }
        }
      }
      double rowmax = 0.0;
      for (size_t t = 0; t < acc.size(); ++t)
        if (present[t]) {
          ++structural;
          rowmax = std::max(rowmax, std::fabs(acc[t]));
        }
      const double thr = drop_rel * rowmax;
      auto kept = [&](size_t t) { return present[t] && acc[t] != 0.0 && std::fabs(acc[t]) > thr; };
      auto wdof = [&](int kc) {
        return kc < nc ? (int32_t)cols[kc] : (int32_t)(N + redges[kc - nc]);
      };
      for (int jb = 0; jb < nc; ++jb) {
        col.push_back(cols[jb]);
        kval.push_back(kacc[jb]);
        mval.push_back(macc[jb]);
        for (int kc = 0; kc < nw; ++kc) {
          const size_t t = (size_t)jb * nw + kc;
          if (kept(t)) {
            kA.push_back(wdof(kc));
            kRel.push_back((uint16_t)kc);
            vA.push_back(acc[t]);
          }
        }
        kptrA.push_back((int32_t)kA.size());
      }
      for (int kc = 0; kc < nw; ++kc) {
        wcol.push_back(wdof(kc));
        if (kc < nc) {
          wpl.push_back((uint16_t)kc);
          wql.push_back((uint16_t)kc);
        } else {
          const int64_t key = ekeys[redges[kc - nc]];
          wpl.push_back((uint16_t)lidx((int32_t)(key / N)));
          wql.push_back((uint16_t)lidx((int32_t)(key % N)));
        }
        for (int jb = 0; jb < nc; ++jb) {
          const size_t t = (size_t)jb * nw + kc;
          if (kept(t)) {
            jB.push_back(cols[jb]);
            jRel.push_back((uint16_t)jb);
            vB.push_back(acc[t]);
          }
        }
        jptrB.push_back((int32_t)jB.size());
      }
      if (col.size() >= (size_t)INT32_MAX || kA.size() >= (size_t)INT32_MAX || jB.size() >= (size_t)INT32_MAX ||
          wcol.size() >= (size_t)INT32_MAX)
        return fail(EGFEM_ERR_SHAPE, "more than 2^31 slots or tensor entries");
      wrowptr[i + 1] = (int32_t)wcol.size();
      rowptr[i + 1] = (int32_t)col.size();
      continue;
    }
    acc.assign((size_t)nc * nc, 0.0);
    present.assign((size_t)nc * nc, 0);
    kacc.assign(nc, 0.0);
    macc.assign(nc, 0.0);
    for (int64_t q = nptr[i]; q < nptr[i + 1]; ++q) {
      const int64_t e = ncell[q];
      const int32_t* c = cells + e * nl;
      const Geom& g = geo[e];
      int a = 0;
      while (c[a] != (int32_t)i) ++a;
      int loc[4];
      for (int b = 0; b < nl; ++b) loc[b] = lidx(c[b]);
      // sum_d d_d lambda_a (convection form); a sum that vanishes in exact
      // arithmetic (e.g. the middle vertices of a Kuhn tetrahedron) is set to
      // zero instead of keeping its rounding noise
      double gsum = 0.0, gabs = 0.0;
      for (int r = 0; r < dim; ++r) {
        gsum += g.G[a][r];
        gabs += std::fabs(g.G[a][r]);
      }
      if (std::fabs(gsum) <= 1e-12 * gabs) gsum = 0.0;
      for (int b = 0; b < nl; ++b) {
        double gg = 0.0;
        for (int r = 0; r < dim; ++r) gg += g.G[a][r] * g.G[b][r];
        const double kab = g.vol * gg;
        kacc[loc[b]] += kab;
        macc[loc[b]] += g.vol * (a == b ? m2_diag : m2_off);
        for (int cc = 0; cc < nl; ++cc) {
          double val;
          if (form == EGFEM_FORM_STIFF) {
            val = kab / (double)(dim + 1);
          } else if (form == EGFEM_FORM_MASS) {
            const int same = (a == b) + (a == cc) + (b == cc);
            val = g.vol * (same == 3 ? m3_aaa : (same == 1 ? m3_aab : m3_abc));
          } else {
            val = gsum * g.vol * (b == cc ? m2_diag : m2_off);
          }
          const size_t idx = (size_t)loc[b] * nc + loc[cc];
          acc[idx] += val;
          present[idx] = 1;
        }
      }
    }
    double rowmax = 0.0;
    for (size_t t = 0; t < acc.size(); ++t)
      if (present[t]) {
        ++structural;
        rowmax = std::max(rowmax, std::fabs(acc[t]));
      }
    const double thr = drop_rel * rowmax;
    auto kept = [&](size_t t) { return present[t] && acc[t] != 0.0 && std::fabs(acc[t]) > thr; };
    for (int jb = 0; jb < nc; ++jb) {
      col.push_back(cols[jb]);
      kval.push_back(kacc[jb]);
      mval.push_back(macc[jb]);
      for (int kc = 0; kc < nc; ++kc) {
        const size_t t = (size_t)jb * nc + kc;
        if (kept(t)) {
          kA.push_back(cols[kc]);
          kRel.push_back((uint16_t)kc);
          vA.push_back(acc[t]);
        }
      }
      kptrA.push_back((int32_t)kA.size());
      if (sym) {
        // half fiber (T_ijk = T_ikj): k at or after j in the row, diagonal halved
        for (int kc = jb; kc < nc; ++kc) {
          const size_t t = (size_t)jb * nc + kc;
          if (kept(t)) {
            hRel.push_back((uint16_t)kc);
            vH.push_back(kc == jb ? 0.5 * acc[t] : acc[t]);
          }
        }
        kptrH.push_back((int32_t)vH.size());
      }
      if (!sym) {
        // B fiber of slot (i, cols[jb]) as k: j runs over the row's columns
        for (int jj = 0; jj < nc; ++jj) {
          const size_t t = (size_t)jj * nc + jb;
          if (kept(t)) {
            jB.push_back(cols[jj]);
            jRel.push_back((uint16_t)jj);
            vB.push_back(acc[t]);
          }
        }
        jptrB.push_back((int32_t)jB.size());
      }
    }
    if (col.size() >= (size_t)INT32_MAX || kA.size() >= (size_t)INT32_MAX)
      return fail(EGFEM_ERR_SHAPE, "more than 2^31 slots or tensor entries");
    rowptr[i + 1] = (int32_t)col.size();
  }
  const int64_t slots = (int64_t)col.size();

  // --- transpose permutation and diagonal ---------------------------------
  std::vector<int32_t> tperm(slots), diag(N);
  for (int64_t i = 0; i < N; ++i) {
    for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s) {
      const int32_t j = col[s];
      const int32_t* b = col.data() + rowptr[j];
      const int32_t* e = col.data() + rowptr[j + 1];
      const int32_t* f = std::lower_bound(b, e, (int32_t)i);
      if (f == e || *f != (int32_t)i) return fail(EGFEM_ERR_MESH, "non-symmetric adjacency");
      tperm[s] = (int32_t)(f - col.data());
      if (j == (int32_t)i) diag[i] = s;
    }
  }

  // --- row blocks --------------------------------------------------------
  const std::vector<int32_t>& kpB = sym ? kptrA : jptrB;
  std::vector<int32_t> blk(1, 0);
  {
    int64_t r0 = 0;
    while (r0 < N) {
      int64_t r1 = r0;
      while (r1 < N) {
        const int64_t rows = r1 + 1 - r0;
        const int64_t sl = rowptr[r1 + 1] - rowptr[r0];
        const int64_t na = kptrA[rowptr[r1 + 1]] - kptrA[rowptr[r0]];
        const int64_t nb = w2 ? jptrB[wrowptr[r1 + 1]] - jptrB[wrowptr[r0]]
                              : kpB[rowptr[r1 + 1]] - kpB[rowptr[r0]];
        const int64_t nw = w2 ? wrowptr[r1 + 1] - wrowptr[r0] : 0;
        if (rows > kCapRows || sl > kCapSlots || na > kCapNnz || nb > kCapNnz || nw > kCapWSlots) break;
        ++r1;
      }
      if (r1 == r0) return fail(EGFEM_ERR_SHAPE, "a node row exceeds the row-block capacity "
                                                 "(1024 tensor entries / 512 slots / 1024 W-slots)");
      blk.push_back((int32_t)r1);
      r0 = r1;
    }
  }

  // Every k of row i's A entries (and every j of its B entries) is a column
  // of row i, so an entry can name it by the block-relative slot of (i, k):
  // 16 bits (at most kCapSlots slots per block).  The stages then gather
  // per slot, not per entry.
  std::vector<uint16_t> kS(kA.size());
  // fiber starts relative to the block's first entry (at most kCapNnz)
  std::vector<uint16_t> kpS((size_t)slots + 1), jpS(sym ? 0 : (size_t)slots + 1);
  // Without the (j, k) symmetry the B stream holds the A entries again: entry
  // (i, j, k) sits in the B fiber of (i, k) (a slot, or a W-slot for
  // W_h != P1), j in column order.  The Jacobian reads, per A entry, the
  // block-relative B position of the same entry (16 bits) instead of the B
  // values and slots, and places the A entry's product there; checked here to
  // be a bijection onto the B stream with bitwise equal values.
  std::vector<uint16_t> bS(sym ? 0 : kA.size());
  std::vector<int32_t> taken;   // B entries of every fiber of the row handed out so far
  // A entry p of the row's j-th slot, in the B fiber fb (the row's kr-th):
  // its B position relative to the block's first B entry pb0
  auto bpos = [&](int32_t p, int32_t fb, int32_t kr, int32_t j, int32_t pb0) {
    const int32_t q = jptrB[fb] + taken[(size_t)kr]++;
    if (q >= jptrB[fb + 1] || jRel[q] != j || std::memcmp(&vB[q], &vA[p], sizeof(double)) != 0) return false;
    bS[p] = (uint16_t)(q - pb0);
    return true;
  };
  auto bad_b = [&]() { return fail(EGFEM_ERR_SHAPE, "internal: the B stream is not a permutation of the A stream"); };
  // W_h = P2: an A entry names its k by the block-relative W-slot of (i, k);
  // the B stream is aligned to W-slots; every W-slot records the block-relative
  // slots of its two endpoints (p | q << 16; p == q for a vertex dof)
  const int64_t wslots = w2 ? (int64_t)wcol.size() : 0;
  std::vector<uint32_t> wpq, wpq2;
  std::vector<int32_t> wmeta;
  if (w2) {
    jpS.assign((size_t)wslots + 1, 0);
    wpq.assign((size_t)wslots, 0);
    if (wq || wcell) wpq2.assign((size_t)wslots, 0);
    wmeta.assign((blk.size() - 1) * 2, 0);
    for (size_t b = 0; b + 1 < blk.size(); ++b) {
      const int32_t s0 = rowptr[blk[b]], w0 = wrowptr[blk[b]];
      wmeta[2 * b] = w0;
      wmeta[2 * b + 1] = wrowptr[blk[b + 1]];
      for (int32_t s = s0; s < rowptr[blk[b + 1]]; ++s) kpS[s] = (uint16_t)(kptrA[s] - kptrA[s0]);
      for (int32_t w = w0; w < wrowptr[blk[b + 1]]; ++w) jpS[w] = (uint16_t)(jptrB[w] - jptrB[w0]);
      for (int32_t i = blk[b]; i < blk[b + 1]; ++i) {
        const int32_t vb = rowptr[i] - s0, wb = wrowptr[i] - w0;
        taken.assign((size_t)(wrowptr[i + 1] - wrowptr[i]), 0);
        for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s)
          for (int32_t p = kptrA[s]; p < kptrA[s + 1]; ++p) {
            kS[p] = (uint16_t)(wb + kRel[p]);
            if (!bpos(p, wrowptr[i] + kRel[p], kRel[p], s - rowptr[i], jptrB[w0])) return bad_b();
          }
        for (int32_t w = wrowptr[i]; w < wrowptr[i + 1]; ++w) {
          wpq[w] = (uint32_t)(vb + wpl[w]) | ((uint32_t)(vb + wql[w]) << 16);
          if (wq || wcell) wpq2[w] = (uint32_t)(vb + wpl2[w]) | ((uint32_t)(vb + wql2[w]) << 16);
        }
      }
    }
  }
  for (size_t b = 0; !w2 && b + 1 < blk.size(); ++b) {
    const int32_t s0 = rowptr[blk[b]];
    for (int32_t s = s0; s < rowptr[blk[b + 1]]; ++s) {
      kpS[s] = (uint16_t)(kptrA[s] - kptrA[s0]);
      if (!sym) jpS[s] = (uint16_t)(jptrB[s] - jptrB[s0]);
    }
    for (int32_t i = blk[b]; i < blk[b + 1]; ++i) {
      const int32_t base = rowptr[i] - s0;
      for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s)
        for (int32_t p = kptrA[s]; p < kptrA[s + 1]; ++p) kS[p] = (uint16_t)(base + kRel[p]);
      if (sym) continue;
      taken.assign((size_t)(rowptr[i + 1] - rowptr[i]), 0);
      for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s)
        for (int32_t p = kptrA[s]; p < kptrA[s + 1]; ++p)
          if (!bpos(p, rowptr[i] + kRel[p], kRel[p], s - rowptr[i], jptrB[s0])) return bad_b();
    }
  }

  // half stream: block-relative k slots and fiber starts, per-block range
  std::vector<uint16_t> kSH, kpSH;
  std::vector<int32_t> hmeta;
  if (sym) {
    kSH.resize(vH.size());
    kpSH.resize((size_t)slots + 1);
    hmeta.resize((blk.size() - 1) * 2);
    for (size_t b = 0; b + 1 < blk.size(); ++b) {
      const int32_t s0 = rowptr[blk[b]], s1 = rowptr[blk[b + 1]];
      hmeta[2 * b] = kptrH[s0];
      hmeta[2 * b + 1] = kptrH[s1];
      for (int32_t s = s0; s < s1; ++s) kpSH[s] = (uint16_t)(kptrH[s] - kptrH[s0]);
      for (int32_t i = blk[b]; i < blk[b + 1]; ++i) {
        const int32_t base = rowptr[i] - s0;
        for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s)
          for (int32_t p = kptrH[s]; p < kptrH[s + 1]; ++p) kSH[p] = (uint16_t)(base + hRel[p]);
      }
    }
  }

  // per-block bounds in one 32-byte record, so that a block's stream loads
  // wait on a single (scalar) load instead of three dependent ones
  std::vector<int32_t> meta((blk.size() - 1) * 8);
  for (size_t b = 0; b + 1 < blk.size(); ++b) {
    const int32_t r0 = blk[b], r1 = blk[b + 1];
    const int32_t s0 = rowptr[r0], s1 = rowptr[r1];
    int32_t* m = meta.data() + 8 * b;
    m[0] = r0;
    m[1] = r1;
    m[2] = s0;
    m[3] = s1;
    m[4] = kptrA[s0];
    m[5] = kptrA[s1];
    m[6] = w2 ? jptrB[wrowptr[r0]] : kpB[s0];
    m[7] = w2 ? jptrB[wrowptr[r1]] : kpB[s1];
  }

  // --- upload -------------------------------------------------------------
  egfem_tensor_s* T = new egfem_tensor_s();
  T->dim = dim;
  T->form = form;
  T->symmetric = sym ? 1 : 0;
  T->n = N;
  T->n_cells = n_cells;
  T->nnz = (int64_t)vA.size();
  T->nnz_b = T->nnz;
  T->structural = structural;
  T->slots = slots;
  T->max_row_slots = max_row_slots;
  // rows wider than the register-held 8 entries (3D meshes) run the 1024-thread
  // resident form, whose Chebyshev steps cost more per step: 6 steps by
  // default there (3D 64^3 with EW forcing: forward 7.04 -> 6.74 ms, adjoint 4.55 -> 4.69 ms)
  if (max_row_slots > kResidentRow) T->krylov_precond = 6;
  int lanes = 4;
  while (lanes < max_row_slots && lanes < 64) lanes *= 2;
  T->lanes_per_row = lanes;
  int klanes = 4;
  while (2 * klanes < max_row_slots && klanes < 64) klanes *= 2;
  T->krylov_lanes = klanes;
  T->krylov_rs = row_shape_for(max_row_slots, klanes);
  T->row_blocks = (int64_t)blk.size() - 1;
  T->w2 = wcell ? 3 : (w2 ? (wq ? 2 : 1) : 0);
  T->n_w = (wq || wcell) ? n_cells * nq : (w2 ? N + (int64_t)ekeys.size() : N);
  T->nq = nq;
  T->wslots = wslots;
  T->max_row_wslots = w2 ? max_row_wslots : max_row_slots;
  T->h_rowptr = rowptr;
  T->h_col = col;
  T->h_coords.assign(coords, coords + (size_t)N * dim);
  hipGetDevice(&T->device);
  int64_t bytes = 0;
  int rc = EGFEM_OK;
  if (rc == EGFEM_OK) rc = upload(rowptr, &T->rowptr, &bytes);
  if (rc == EGFEM_OK) rc = upload(col, &T->col, &bytes);
  if (rc == EGFEM_OK) rc = upload(diag, &T->diag, &bytes);
  if (rc == EGFEM_OK) rc = upload(tperm, &T->tperm, &bytes);
  if (rc == EGFEM_OK) rc = upload(kptrA, &T->kptrA, &bytes);
  if (rc == EGFEM_OK) rc = upload(kA, &T->kA, &bytes);
  if (rc == EGFEM_OK) rc = upload(vA, &T->vA, &bytes);
  if (rc == EGFEM_OK) rc = upload(kS, &T->kS, &bytes);
  if (rc == EGFEM_OK && !sym) rc = upload(bS, &T->bS, &bytes);
  if (rc == EGFEM_OK) rc = upload(kpS, &T->kpS, &bytes);
  if (rc == EGFEM_OK && !sym) rc = upload(jpS, &T->jpS, &bytes);
  if (rc == EGFEM_OK && !sym) rc = upload(jptrB, &T->jptrB, &bytes);
  if (rc == EGFEM_OK && !sym) rc = upload(jB, &T->jB, &bytes);
  if (rc == EGFEM_OK && !sym) rc = upload(vB, &T->vB, &bytes);
  if (rc == EGFEM_OK) rc = upload(kval, &T->kval, &bytes);
  if (rc == EGFEM_OK) rc = upload(mval, &T->mval, &bytes);
  if (rc == EGFEM_OK) rc = upload(blk, &T->blk_row, &bytes);
  if (rc == EGFEM_OK) rc = upload(meta, &T->blk_meta, &bytes);
  if (w2) {
    if (rc == EGFEM_OK) rc = upload(wrowptr, &T->wrowptr, &bytes);
    if (rc == EGFEM_OK) rc = upload(wcol, &T->wcol, &bytes);
    if (rc == EGFEM_OK) rc = upload(wpq, &T->wpq, &bytes);
    if (rc == EGFEM_OK) rc = upload(wmeta, &T->wmeta, &bytes);
  }
  if (sym) {
    if (rc == EGFEM_OK) rc = upload(kSH, &T->kSH, &bytes);
    if (rc == EGFEM_OK) rc = upload(vH, &T->vH, &bytes);
    if (rc == EGFEM_OK) rc = upload(kpSH, &T->kpSH, &bytes);
    if (rc == EGFEM_OK) rc = upload(hmeta, &T->hmeta, &bytes);
    T->nnz_h = (int64_t)vH.size();
    T->action_half = 0;   // the autotuner switches to it where it is faster
  }
  if (w2 && !wq && !wcell) {
    // P2: the endpoints of every edge dof (Pi_u u at the edge midpoints)
    std::vector<int32_t> ep(ekeys.size() * 2);
    for (size_t t = 0; t < ekeys.size(); ++t) {
      ep[2 * t] = (int32_t)(ekeys[t] / N);
      ep[2 * t + 1] = (int32_t)(ekeys[t] % N);
    }
    if (rc == EGFEM_OK) rc = upload(ep, &T->p2_edges, &bytes);
  }
  if (wq || wcell) {
    // vertex ids of every cell (padded to 4 with the first): the points of
    // W_h = I_k evaluate Pi_u u from them, W_h = P0 its gradient
    std::vector<int32_t> c4((size_t)n_cells * 4);
    for (int64_t e = 0; e < n_cells; ++e) {
      const int32_t* c = cells + e * nl;
      for (int m = 0; m < 4; ++m) c4[4 * e + m] = c[m < nl ? m : 0];
    }
    int32_t* d4 = nullptr;
    if (rc == EGFEM_OK) rc = upload(c4, &d4, &bytes);
    T->e_cell4 = reinterpret_cast<int4*>(d4);
  }
  if (wcell) {
    // the gradient interpolation: grad lambda_m (4 x 3 doubles, zero padded)
    // of every cell
    std::vector<double> gr((size_t)n_cells * 12, 0.0);
    for (int64_t e = 0; e < n_cells; ++e)
      for (int m = 0; m < nl; ++m)
        for (int r = 0; r < dim; ++r) gr[12 * e + 3 * m + r] = geo[e].G[m][r];
    if (rc == EGFEM_OK) rc = upload(gr, &T->e_grad, &bytes);
    if (rc == EGFEM_OK) rc = hipMalloc((void**)&T->e_acoef, (size_t)n_cells * sizeof(double)) == hipSuccess
                                ? EGFEM_OK : fail(EGFEM_ERR_OOM, "hipMalloc of the cell coefficients failed");
    if (rc == EGFEM_OK) rc = hipMalloc((void**)&T->e_wv, (size_t)n_cells * 4 * sizeof(double)) == hipSuccess
                                ? EGFEM_OK : fail(EGFEM_ERR_OOM, "hipMalloc of the cell weights failed");
    bytes += n_cells * 5 * (int64_t)sizeof(double);
  }
  if (wq || wcell) {
    std::vector<double> ql(16, 0.0);
    for (int q = 0; q < nq; ++q)
      for (int m = 0; m < 4; ++m) ql[4 * q + m] = qlam[q][m];
    if (rc == EGFEM_OK) rc = upload(wpq2, &T->wpq2, &bytes);
    if (rc == EGFEM_OK) rc = upload(wqi, &T->wqi, &bytes);
    if (rc == EGFEM_OK) rc = upload(ql, &T->qlam, &bytes);
  }
  if (sym) {
    T->jptrB = T->kptrA;
    T->jB = T->kA;
    T->vB = T->vA;
    T->jpS = T->kpS;
  }
  T->device_bytes = bytes;
  if (rc != EGFEM_OK) {
    egfem_tensor_destroy(T);
    return rc;
  }
  *out = T;
  return EGFEM_OK;
}

}  // namespace

extern "C" int egfem_build_tensor(int dim, int64_t n_nodes, const double* coords, int64_t n_cells,
                                  const int32_t* cells, int form, double drop_rel, egfem_tensor_t* out) {
  return build_impl(dim, n_nodes, coords, n_cells, cells, form, EGFEM_W_P1, drop_rel, out);
}

extern "C" int egfem_build_tensor_w(int dim, int64_t n_nodes, const double* coords, int64_t n_cells,
                                    const int32_t* cells, int form, int wspace, double drop_rel,
                                    egfem_tensor_t* out) {
  return build_impl(dim, n_nodes, coords, n_cells, cells, form, wspace, drop_rel, out);
}

extern "C" int egfem_attach_elements(egfem_tensor_t T, int dim, int64_t n_nodes, const double* coords,
                                     int64_t n_cells, const int32_t* cells) {
  using namespace egfem;
  if (!T || !coords || !cells) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->form != EGFEM_FORM_STIFF || T->w2)
    return fail(EGFEM_ERR_ARG, "the element-factored form exists for the stiffness tensor with W_h = P1");
  if (dim != T->dim || n_nodes != T->n || n_cells != T->n_cells)
    return fail(EGFEM_ERR_SHAPE, "mesh sizes differ from the tensor's");
  if (n_cells >= (int64_t(1) << 29)) return fail(EGFEM_ERR_SHAPE, "too many cells for the incidence encoding");
  const int nl = dim + 1;
  const int kstride = ((nl * (nl + 1) / 2) + 1) & ~1;
  std::vector<int32_t> cell4((size_t)n_cells * 4);
  std::vector<double> kp((size_t)n_cells * kstride, 0.0);
  std::vector<int32_t> nptr(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_cells; ++e) {
    const int32_t* c = cells + e * nl;
    for (int a = 0; a < nl; ++a)
      if (c[a] < 0 || c[a] >= n_nodes) return fail(EGFEM_ERR_MESH, "cell index out of range");
    Geom g;
    if (!cell_geometry(dim, coords, c, g)) return fail(EGFEM_ERR_MESH, "degenerate cell");
    for (int m = 0; m < 4; ++m) cell4[4 * e + m] = c[m < nl ? m : 0];
    int t = 0;
    for (int a = 0; a < nl; ++a)
      for (int b = a; b < nl; ++b) {
        double gg = 0.0;
        for (int r = 0; r < dim; ++r) gg += g.G[a][r] * g.G[b][r];
        kp[(size_t)e * kstride + t++] = g.vol * gg;
      }
    for (int a = 0; a < nl; ++a) nptr[c[a] + 1]++;
  }
  int maxinc = 0;
  for (int64_t i = 0; i < n_nodes; ++i) {
    maxinc = std::max(maxinc, nptr[i + 1]);
    nptr[i + 1] += nptr[i];
  }
  std::vector<int32_t> inc(nptr[n_nodes]);
  {
    std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
    for (int64_t e = 0; e < n_cells; ++e)
      for (int a = 0; a < nl; ++a) inc[fill[cells[e * nl + a]]++] = (int32_t)((e << 2) | a);
  }
  // replace previous data
  for (void* p : {(void*)T->e_cell4, (void*)T->e_kp, (void*)T->e_nptr, (void*)T->e_inc})
    if (p) hipFree(p);
  T->e_cell4 = nullptr;
  T->e_kp = nullptr;
  T->e_nptr = nullptr;
  T->e_inc = nullptr;
  int64_t bytes = 0;
  int32_t* c4 = nullptr;
  int rc = upload(cell4, &c4, &bytes);
  if (rc == EGFEM_OK) rc = upload(kp, &T->e_kp, &bytes);
  if (rc == EGFEM_OK) rc = upload(nptr, &T->e_nptr, &bytes);
  if (rc == EGFEM_OK) rc = upload(inc, &T->e_inc, &bytes);
  T->e_cell4 = reinterpret_cast<int4*>(c4);
  if (rc != EGFEM_OK) return rc;
  int lanes = 2;
  while (lanes < maxinc && lanes < 64) lanes *= 2;
  T->e_lanes = lanes;
  T->e_kstride = kstride;
  T->e_cells = n_cells;
  T->device_bytes += bytes;
  return EGFEM_OK;
}


// Unique storage of the fully symmetric P1 mass tensor T_ijk = int phi_i phi_j phi_k:
// one value per index multiset, i.e. T_iii per vertex, T_aab and T_abb per edge
// (a < b) and T_abc per face of the mesh (three distinct vertices of one cell),
// N + 2E + F values against N + 6E + 6F stored entries of the full stream.
extern "C" int egfem_attach_unique(egfem_tensor_t T, int dim, int64_t n_nodes, const double* coords,
                                   int64_t n_cells, const int32_t* cells, int64_t* n_unique) {
  using namespace egfem;
  if (!T || !coords || !cells) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->form != EGFEM_FORM_MASS || T->w2)
    return fail(EGFEM_ERR_ARG, "the unique storage exists for the fully symmetric mass tensor with W_h = P1");
  if (dim != T->dim || n_nodes != T->n || n_cells != T->n_cells)
    return fail(EGFEM_ERR_SHAPE, "mesh sizes differ from the tensor's");
  const int nl = dim + 1;
  const int64_t N = n_nodes;
  for (int64_t e = 0; e < n_cells * nl; ++e)
    if (cells[e] < 0 || cells[e] >= N) return fail(EGFEM_ERR_MESH, "cell index out of range");
  // edges (min * N + max) and faces (sorted vertex triples) of the cells
  std::vector<int64_t> ekeys;
  std::vector<std::array<int32_t, 3>> faces;
  ekeys.reserve((size_t)n_cells * nl * dim / 2);
  for (int64_t e = 0; e < n_cells; ++e) {
    const int32_t* c = cells + e * nl;
    for (int a = 0; a < nl; ++a)
      for (int b = a + 1; b < nl; ++b) {
        ekeys.push_back(std::min<int64_t>(c[a], c[b]) * N + std::max<int64_t>(c[a], c[b]));
        for (int m = b + 1; m < nl; ++m) {
          std::array<int32_t, 3> f = {c[a], c[b], c[m]};
          std::sort(f.begin(), f.end());
          faces.push_back(f);
        }
      }
  }
  std::sort(ekeys.begin(), ekeys.end());
  ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
  std::sort(faces.begin(), faces.end());
  faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
  const int64_t E = (int64_t)ekeys.size(), F = (int64_t)faces.size();
  if (E >= (int64_t(1) << 30) || F >= (int64_t(1) << 31))
    return fail(EGFEM_ERR_SHAPE, "too many edges or faces for the unique storage");
  // every multiset appears in the full stream once per distinct ordering
  if (N + 6 * E + 6 * F != T->nnz)
    return fail(EGFEM_ERR_SHAPE, "the mesh does not match the tensor's entries");
  auto edge_of = [&](int64_t x, int64_t y) {
    const int64_t key = std::min(x, y) * N + std::max(x, y);
    return (int64_t)(std::lower_bound(ekeys.begin(), ekeys.end(), key) - ekeys.begin());
  };
  auto face_of = [&](std::array<int32_t, 3> f) {
    std::sort(f.begin(), f.end());
    return (int64_t)(std::lower_bound(faces.begin(), faces.end(), f) - faces.begin());
  };
  const int64_t foff = N + 2 * E;
  std::vector<double> val((size_t)(foff + F), 0.0);
  for (int64_t e = 0; e < n_cells; ++e) {
    const int32_t* c = cells + e * nl;
    Geom g;
    if (!cell_geometry(dim, coords, c, g)) return fail(EGFEM_ERR_MESH, "degenerate cell");
    for (int a = 0; a < nl; ++a) {
      int x[4] = {0, 0, 0, 0};
      x[a] = 3;
      val[c[a]] += g.vol * mono(dim, x);
      for (int b = a + 1; b < nl; ++b) {
        const int lo = c[a] < c[b] ? a : b, hi = c[a] < c[b] ? b : a;
        const int64_t eid = edge_of(c[a], c[b]);
        int y[4] = {0, 0, 0, 0};
        y[lo] = 2;
        y[hi] = 1;
        val[N + 2 * eid] += g.vol * mono(dim, y);      // T_{lo lo hi}
        int z[4] = {0, 0, 0, 0};
        z[lo] = 1;
        z[hi] = 2;
        val[N + 2 * eid + 1] += g.vol * mono(dim, z);  // T_{lo hi hi}
        for (int m = b + 1; m < nl; ++m) {
          int w[4] = {0, 0, 0, 0};
          w[a] = w[b] = w[m] = 1;
          val[foff + face_of({c[a], c[b], c[m]})] += g.vol * mono(dim, w);
        }
      }
    }
  }
  // slot references: the edge of every off-diagonal slot, with its orientation
  const std::vector<int32_t>& rp = T->h_rowptr;
  const std::vector<int32_t>& cl = T->h_col;
  std::vector<int32_t> sref((size_t)T->slots, -1);
  for (int64_t i = 0; i < N; ++i)
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
      if (cl[p] != i) {
        const int64_t eid = edge_of(i, cl[p]);
        if (eid >= E || ekeys[eid] != std::min<int64_t>(i, cl[p]) * N + std::max<int64_t>(i, cl[p]))
          return fail(EGFEM_ERR_SHAPE, "the mesh does not match the tensor's pattern");
        sref[p] = (int32_t)(2 * eid + (i > cl[p] ? 1 : 0));
      }
  // face references of every row, in face order
  std::vector<int32_t> fptr(N + 1, 0);
  for (const auto& f : faces)
    for (int v = 0; v < 3; ++v) fptr[f[v] + 1]++;
  int max_faces = 0;
  for (int64_t i = 0; i < N; ++i) {
    max_faces = std::max(max_faces, fptr[i + 1]);
    fptr[i + 1] += fptr[i];
  }
  std::vector<int32_t> fref((size_t)2 * fptr[N]);
  {
    std::vector<int32_t> fill(fptr.begin(), fptr.end() - 1);
    auto local = [&](int64_t i, int32_t j) {
      const auto b = cl.begin() + rp[i], en = cl.begin() + rp[i + 1];
      const auto it = std::lower_bound(b, en, j);
      return (it != en && *it == j) ? (int)(it - b) : -1;
    };
    for (int64_t t = 0; t < F; ++t)
      for (int v = 0; v < 3; ++v) {
        const int32_t i = faces[t][v], j = faces[t][(v + 1) % 3], k = faces[t][(v + 2) % 3];
        const int sj = local(i, j), sk = local(i, k);
        if (sj < 0 || sk < 0) return fail(EGFEM_ERR_SHAPE, "the mesh does not match the tensor's pattern");
        const int32_t q = fill[i]++;
        fref[2 * (size_t)q] = (int32_t)t;
        fref[2 * (size_t)q + 1] = sj | (sk << 16);
      }
  }
  if (T->max_row_slots > 512) return fail(EGFEM_ERR_SHAPE, "rows of more than 512 slots");
  // replace previous data
  for (void* p : {(void*)T->u_val, (void*)T->u_sref, (void*)T->u_fptr, (void*)T->u_fref})
    if (p) hipFree(p);
  T->u_val = nullptr;
  T->u_sref = nullptr;
  T->u_fptr = nullptr;
  T->u_fref = nullptr;
  int64_t bytes = 0;
  int32_t* fr = nullptr;
  int rc = upload(val, &T->u_val, &bytes);
  if (rc == EGFEM_OK) rc = upload(sref, &T->u_sref, &bytes);
  if (rc == EGFEM_OK) rc = upload(fptr, &T->u_fptr, &bytes);
  if (rc == EGFEM_OK) rc = upload(fref, &fr, &bytes);
  T->u_fref = reinterpret_cast<int2*>(fr);
  if (rc != EGFEM_OK) return rc;
  // lanes per row from the row's slot count (2D: 4, 3D Kuhn meshes: 8; the
  // face references are read in several passes)
  const int stride = std::max(T->max_row_slots, 1);
  int lanes = 2;
  while (2 * lanes < stride && lanes < 64) lanes *= 2;
  // the rows of a workgroup stage u and a of their slots in at most 32 KB of LDS
  while ((size_t)(kBlockThreads / lanes) * stride * 16 > 32768 && lanes < 64) lanes *= 2;
  T->u_lanes = lanes;
  T->u_stride = stride;
  T->u_count = foff + F;
  T->u_foff = foff;
  T->device_bytes += bytes;
  if (n_unique) *n_unique = T->u_count;
  return EGFEM_OK;
}
