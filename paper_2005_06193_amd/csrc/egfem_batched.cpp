// Batched Newton entry point.
#include "egfem_internal.h"

extern "C" int egfem_newton_batched(int count, const egfem_tensor_t* Ts, const egfem_problem* ps,
                                    double* const* us, const egfem_newton_opts* o,
                                    egfem_newton_stats* stats, void* stream) {
  using namespace egfem;
  if (count <= 0 || !Ts || !ps || !us) return fail(EGFEM_ERR_ARG, "null argument or count <= 0");
  int worst = EGFEM_OK;
  for (int m = 0; m < count; ++m) {
    const int rc = egfem_newton(Ts[m], &ps[m], us[m], o, stats ? &stats[m] : nullptr, stream);
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
  }
  return worst;
}
