// Host driver for the CPU tests of the compact row partition: reads a mesh
// graph (dimension and node count, coordinates, CSR row pointers and columns)
// from binary files, runs the library's partition into G parts and writes the
// result back (part offsets, row list, part-local column positions, neighbour
// lists, largest part).  Built with g++ against the library's partition source.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2005_06193_amd/csrc/egfem_internal.h"

namespace egfem {
void set_error(const std::string& msg) { std::fprintf(stderr, "%s\n", msg.c_str()); }
int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}
}  // namespace egfem

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
static bool write_all(const std::string& path, const std::vector<T>& v) {
  FILE* fp = std::fopen(path.c_str(), "wb");
  if (!fp) return false;
  const bool ok = v.empty() || std::fwrite(v.data(), sizeof(T), v.size(), fp) == v.size();
  std::fclose(fp);
  return ok;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s PREFIX G\n", argv[0]);
    return 2;
  }
  const std::string p = argv[1];
  const int G = std::atoi(argv[2]);
  std::vector<int64_t> hdr;
  std::vector<double> X;
  std::vector<int32_t> rowptr, col;
  if (!read_all(p + ".hdr", hdr) || hdr.size() != 2 || !read_all(p + ".x", X) || !read_all(p + ".rp", rowptr) ||
      !read_all(p + ".col", col)) {
    std::fprintf(stderr, "cannot read %s.*\n", p.c_str());
    return 2;
  }
  const int dim = (int)hdr[0];
  const int64_t n = hdr[1];
  if ((int64_t)rowptr.size() != n + 1 || (int64_t)X.size() != n * dim || (int64_t)col.size() != rowptr[n]) {
    std::fprintf(stderr, "inconsistent mesh graph files\n");
    return 2;
  }
  // optional mask of rows left out (the free-row partition)
  std::vector<uint8_t> skip;
  const bool has_skip = read_all(p + ".skip", skip);
  if (has_skip && (int64_t)skip.size() != n) {
    std::fprintf(stderr, "inconsistent skip mask\n");
    return 2;
  }
  egfem::CompactPartition cp;
  const int rc = egfem::make_compact_partition(dim, X.data(), n, rowptr.data(), col.data(), G, cp,
                                               has_skip ? skip.data() : nullptr);
  std::printf("rc %d\n", rc);
  if (rc != EGFEM_OK) return 0;
  const std::vector<int32_t> meta = {cp.maxrows, egfem::kMaxNbrLists};
  const bool ok = write_all(p + ".kr", cp.kr) && write_all(p + ".rlist", cp.rlist) &&
                  write_all(p + ".kloc", cp.kloc) && write_all(p + ".nbr", cp.nbr) && write_all(p + ".meta", meta);
  return ok ? 0 : 2;
}
