// Problem residual and its norm for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid allocation): the same residual kernel as egfem_problem_residual, with
// its per-workgroup partial sums of F_i^2 in a fixed-size array of this
// library instead of the handle's workspace, and their total formed on the
// device.  No hipMalloc, hipFree or allocating call on any path.
#include <cmath>
#include <mutex>

#include "egfem_internal.h"

namespace egfem {
namespace {

// Partial sums the array holds (the residual kernel writes one per workgroup
// run, i.e. per row block of an untuned handle or per run of an autotuned one).
constexpr int64_t kNoAllocMaxRuns = 16384;
constexpr int kNoAllocMaxDevices = 64;

// [0, kNoAllocMaxRuns): partial sums; [kNoAllocMaxRuns]: their total.  Every
// device the library runs on holds its own copy until the process ends.  In
// host code this name is not a device address: kernels and copies use the
// address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) double scratch[kNoAllocMaxRuns + 32];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(double** out) {
  int dev = -1;
  EGFEM_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(EGFEM_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(EGFEM_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return EGFEM_OK;
}

// out[0] = sum of part[0, n): thread t adds entries t, t + 256, ... in order,
// then a fixed-order tree over the 256 thread sums (deterministic).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int64_t n,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) s += part[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace
}  // namespace egfem

extern "C" int egfem_problem_residual_noalloc(egfem_tensor_t T, const egfem_problem* p, const double* u,
                                              double* F, double* norm, void* stream) {
  using namespace egfem;
  if (!T || !p || !u || !F) return fail(EGFEM_ERR_ARG, "null argument");
  if (T->w2 == 3) return fail(EGFEM_ERR_ARG, "W_h = P0 handles take the gradient coefficient (egfem_picard_grad)");
  if (F == u) return fail(EGFEM_ERR_ARG, "F must not alias u");
  int dev = -1;
  EGFEM_HIP_CHECK(hipGetDevice(&dev));
  if (dev != T->device) return fail(EGFEM_ERR_ARG, "the handle's device must be the current device");
  const int64_t nrun = action_runs(T);
  if (nrun > kNoAllocMaxRuns)
    return fail(EGFEM_ERR_SHAPE, "the residual kernel of this handle writes " + std::to_string(nrun) +
                                     " partial sums, more than the " + std::to_string(kNoAllocMaxRuns) +
                                     " the no-allocation array holds (tune the action runs or use "
                                     "egfem_problem_residual)");
  double* scr = nullptr;
  int rc = scratch_address(&scr);
  if (rc != EGFEM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const ProblemView pv{p->a0, p->a0_const, p->load, p->dirichlet, p->add_stiffness};
  EGFEM_HIP_CHECK(launch_action_problem(T, pv, u, nullptr, 0.0, nullptr, F, scr, st));
  if (!norm) return EGFEM_OK;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, scr, nrun, scr + kNoAllocMaxRuns);
  EGFEM_HIP_CHECK(hipGetLastError());
  double sq = 0.0;
  EGFEM_HIP_CHECK(hipMemcpyAsync(&sq, scr + kNoAllocMaxRuns, sizeof(double), hipMemcpyDeviceToHost, st));
  EGFEM_HIP_CHECK(hipStreamSynchronize(st));
  *norm = std::sqrt(sq);
  return EGFEM_OK;
}
