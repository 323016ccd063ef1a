// Streaming-read ceiling: the bandwidth a plain read of device memory reaches
// with the launch arrangement of the tensor action (one contiguous chunk per
// workgroup, every load of a thread issued before the first is used, chunks
// mapped to the XCDs in contiguous regions).  It is the measured reference the
// tensor action's HBM fraction is read against; it computes one sum per chunk.
#include "egfem_internal.h"

namespace egfem {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeVec = 4;                                   // 16-byte loads per thread
constexpr int64_t kProbeChunk = int64_t(kProbeThreads) * kProbeVec * 2;   // doubles per workgroup

__device__ __forceinline__ int64_t probe_block(int64_t bid, int64_t nblk) {
  const int64_t per = (nblk + 7) >> 3;
  const int64_t lb = (bid & 7) * per + (bid >> 3);
  return lb < nblk ? lb : -1;
}

// partial[c] = sum of x[c * kProbeChunk, min(n, (c + 1) * kProbeChunk)), each
// thread's kProbeVec 16-byte loads strided by the workgroup width (coalesced)
__global__ __launch_bounds__(kProbeThreads) void k_stream_read(const double* __restrict__ x, int64_t n,
                                                              int64_t nchunk, double* __restrict__ partial) {
  __shared__ double sh[kProbeThreads / 64];
  const int64_t c = probe_block(blockIdx.x, nchunk);
  if (c < 0) return;
  const int64_t base = c * kProbeChunk;
  const int64_t len = n - base < kProbeChunk ? n - base : kProbeChunk;
  double acc = 0.0;
  if (len == kProbeChunk && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    const double2* x2 = reinterpret_cast<const double2*>(x + base);
    double2 v[kProbeVec];
#pragma unroll
    for (int q = 0; q < kProbeVec; ++q) v[q] = x2[threadIdx.x + q * kProbeThreads];
#pragma unroll
    for (int q = 0; q < kProbeVec; ++q) acc += v[q].x + v[q].y;
  } else {
    for (int64_t t = threadIdx.x; t < len; t += kProbeThreads) acc += x[base + t];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kProbeThreads / 64; ++w) s += sh[w];
    partial[c] = s;
  }
}

}  // namespace
}  // namespace egfem

extern "C" int64_t egfem_stream_read_chunks(int64_t n) {
  return n <= 0 ? 0 : (n + egfem::kProbeChunk - 1) / egfem::kProbeChunk;
}

extern "C" int egfem_stream_read(const double* x, int64_t n, double* partial, int64_t n_partial, void* stream) {
  using namespace egfem;
  if (n < 0 || (n > 0 && (!x || !partial))) return fail(EGFEM_ERR_ARG, "null argument or n < 0");
  const int64_t nchunk = egfem_stream_read_chunks(n);
  if (n_partial < nchunk) return fail(EGFEM_ERR_SHAPE, "partial holds fewer entries than chunks");
  if (nchunk == 0) return EGFEM_OK;
  const int64_t grid = ((nchunk + 7) >> 3) << 3;
  if (grid > INT32_MAX) return fail(EGFEM_ERR_SHAPE, "too many chunks");
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)grid), dim3(kProbeThreads), 0, (hipStream_t)stream, x, n, nchunk,
                     partial);
  EGFEM_HIP_CHECK(hipGetLastError());
  return EGFEM_OK;
}
