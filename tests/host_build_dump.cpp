// Host driver for the CPU tests of the offline tensor build: the library's
// build source (exact element integrals, fiber streams, row blocks, storage
// variants) is compiled with g++ -- with the address and undefined-behaviour
// sanitizers in the test -- and linked against a host-memory stand-in for the
// five HIP runtime calls it makes (allocation, copy, fill, free, device
// query), so every "device" array of the handle is ordinary host memory that
// this driver can read back.
//
// Reads a mesh (dim, n_nodes, n_cells, form, wspace; coordinates; cells) from
// binary files, builds the handle, checks the block-relative stream format
// against the global streams, attaches the storage variants where they apply,
// and writes the A stream as COO (i, j, k, v) plus the counts.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2005_06193_amd/csrc/egfem_internal.h"

// ---- host stand-ins of the HIP runtime calls of the build -----------------
hipError_t hipMalloc(void** ptr, size_t size) {
  *ptr = std::calloc(size ? size : 1, 1);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* ptr) {
  std::free(ptr);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (bytes) std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int value, size_t bytes) {
  if (bytes) std::memset(dst, value, bytes);
  return hipSuccess;
}
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}

namespace egfem {
void set_error(const std::string& msg) { std::fprintf(stderr, "%s\n", msg.c_str()); }
int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}
}  // namespace egfem

// The test releases nothing (the process ends; leak detection is off).
extern "C" void egfem_tensor_destroy(egfem_tensor_t) {}

template <class T>
static bool read_all(const std::string& path, std::vector<T>& v) {
  FILE* fp = std::fopen(path.c_str(), "rb");
  if (!fp) return false;
  T x;
  while (std::fread(&x, sizeof(T), 1, fp) == 1) v.push_back(x);
  std::fclose(fp);
  return true;
}

template <class T>
static bool write_all(const std::string& path, const T* v, size_t n) {
  FILE* fp = std::fopen(path.c_str(), "wb");
  if (!fp) return false;
  const bool ok = n == 0 || std::fwrite(v, sizeof(T), n, fp) == n;
  std::fclose(fp);
  return ok;
}

// Every entry of the block-relative streams names the same slot / fiber as
// the global streams: fiber starts and the slot of (i, k) (A); without the
// (j, k) symmetry, the B position of every A entry (i, j, k) lies in the B
// fiber of slot (i, k), names column j, holds the same value bit for bit,
// and no B position is named twice.
static int check_blocks(const egfem_tensor_s* T) {
  const int4* meta = reinterpret_cast<const int4*>(T->blk_meta);
  int bad = 0;
  std::vector<int> hit;
  for (int64_t b = 0; b < T->row_blocks; ++b) {
    const int4 x = meta[2 * b], y = meta[2 * b + 1];
    const int r0 = x.x, r1 = x.y, s0 = x.z, s1 = x.w, pa0 = y.x, pa1 = y.y, pb0 = y.z, pb1 = y.w;
    if (T->blk_row[b] != r0 || T->blk_row[b + 1] != r1 || T->rowptr[r0] != s0 || T->rowptr[r1] != s1) ++bad;
    if (r1 - r0 > egfem::kCapRows || s1 - s0 > egfem::kCapSlots || pa1 - pa0 > egfem::kCapNnz ||
        pb1 - pb0 > egfem::kCapNnz)
      ++bad;
    hit.assign((size_t)(pb1 - pb0), 0);
    for (int i = r0; i < r1; ++i)
      for (int s = T->rowptr[i]; s < T->rowptr[i + 1]; ++s) {
        if (T->kptrA[s] != pa0 + T->kpS[s]) ++bad;
        if (!T->symmetric && T->jptrB[s] != pb0 + T->jpS[s]) ++bad;
        for (int p = T->kptrA[s]; p < T->kptrA[s + 1]; ++p) {
          const int ks = s0 + T->kS[p];
          if (ks < T->rowptr[i] || ks >= T->rowptr[i + 1] || T->col[ks] != T->kA[p]) {
            ++bad;
            continue;
          }
          if (T->symmetric) continue;
          const int q = pb0 + T->bS[p];
          if (q < T->jptrB[ks] || q >= T->jptrB[ks + 1] || T->jB[q] != T->col[s] ||
              std::memcmp(&T->vB[q], &T->vA[p], sizeof(double)) != 0 || hit[q - pb0]++)
            ++bad;
        }
      }
    if (T->kptrA[s1] != pa1) ++bad;
    if (!T->symmetric && pb1 - pb0 != pa1 - pa0) ++bad;
  }
  return bad;
}

// W_h != P1: every A entry names a W-slot of its own row, and its B position
// lies in the B fiber of that W-slot, names the entry's column j, holds the
// same value bit for bit, and is named by no other entry of the block.
static int check_blocks_w(const egfem_tensor_s* T) {
  const int4* meta = reinterpret_cast<const int4*>(T->blk_meta);
  const int2* wm = reinterpret_cast<const int2*>(T->wmeta);
  int bad = 0;
  std::vector<int> hit;
  for (int64_t b = 0; b < T->row_blocks; ++b) {
    const int4 x = meta[2 * b], y = meta[2 * b + 1];
    const int r0 = x.x, r1 = x.y, pa0 = y.x, pa1 = y.y, pb0 = y.z, pb1 = y.w;
    const int w0 = wm[b].x;
    if (pb1 - pb0 != pa1 - pa0 || T->jptrB[w0] != pb0) ++bad;
    hit.assign((size_t)(pb1 - pb0), 0);
    for (int i = r0; i < r1; ++i)
      for (int s = T->rowptr[i]; s < T->rowptr[i + 1]; ++s)
        for (int p = T->kptrA[s]; p < T->kptrA[s + 1]; ++p) {
          const int w = w0 + T->kS[p];
          const int q = pb0 + T->bS[p];
          if (w < T->wrowptr[i] || w >= T->wrowptr[i + 1] || q < T->jptrB[w] || q >= T->jptrB[w + 1] ||
              T->jB[q] != T->col[s] || std::memcmp(&T->vB[q], &T->vA[p], sizeof(double)) != 0 || hit[q - pb0]++)
            ++bad;
        }
  }
  return bad;
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s PREFIX\n", argv[0]);
    return 2;
  }
  const std::string p = argv[1];
  std::vector<int64_t> hdr;
  std::vector<double> X;
  std::vector<int32_t> cells;
  if (!read_all(p + ".hdr", hdr) || hdr.size() != 5 || !read_all(p + ".x", X) || !read_all(p + ".cells", cells)) {
    std::fprintf(stderr, "cannot read %s.*\n", p.c_str());
    return 2;
  }
  const int dim = (int)hdr[0], form = (int)hdr[3], wspace = (int)hdr[4];
  const int64_t n = hdr[1], nc = hdr[2];
  if ((int64_t)X.size() != n * dim || (int64_t)cells.size() != nc * (dim + 1)) {
    std::fprintf(stderr, "inconsistent mesh files\n");
    return 2;
  }
  egfem_tensor_t T = nullptr;
  int rc = egfem_build_tensor_w(dim, n, X.data(), nc, cells.data(), form, wspace, 1e-13, &T);
  std::printf("rc %d\n", rc);
  if (rc != EGFEM_OK) return 0;
  std::printf("nnz %lld slots %lld blocks %lld structural %lld\n", (long long)T->nnz, (long long)T->slots,
              (long long)T->row_blocks, (long long)T->structural);
  if (wspace != EGFEM_W_P1) {   // W_h != P1: built under the sanitizers, B positions checked, no stream dump
    std::printf("block_mismatch %d\n", check_blocks_w(T));
    return 0;
  }
  const int bad = check_blocks(T);
  std::printf("block_mismatch %d\n", bad);
  // storage variants of the same mesh
  if (form == EGFEM_FORM_MASS) {
    int64_t nu = 0;
    std::printf("unique_rc %d %lld\n", egfem_attach_unique(T, dim, n, X.data(), nc, cells.data(), &nu),
                (long long)nu);
  }
  if (form == EGFEM_FORM_STIFF)
    std::printf("elements_rc %d\n", egfem_attach_elements(T, dim, n, X.data(), nc, cells.data()));
  std::vector<int32_t> I(T->nnz), J(T->nnz);
  for (int64_t i = 0; i < n; ++i)
    for (int s = T->rowptr[i]; s < T->rowptr[i + 1]; ++s)
      for (int q = T->kptrA[s]; q < T->kptrA[s + 1]; ++q) {
        I[q] = (int32_t)i;
        J[q] = T->col[s];
      }
  const bool ok = write_all(p + ".i", I.data(), I.size()) && write_all(p + ".j", J.data(), J.size()) &&
                  write_all(p + ".k", T->kA, (size_t)T->nnz) && write_all(p + ".v", T->vA, (size_t)T->nnz);
  return ok ? 0 : 2;
}
