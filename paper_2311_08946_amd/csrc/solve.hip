// BiCGStab solve of C u = r and C^T lambda = g on the device.
#include <hip/hip_runtime.h>

#include "runtime.h"

using namespace pdd;

extern "C" pdd_status pdd_solve_G(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                                  const pdd_solve_opts* opts, void* stream, pdd_solve_info* info) {
  (void)sys; (void)rhs; (void)u; (void)transpose; (void)opts; (void)stream; (void)info;
  return fail(PDD_EINVAL, "pdd_solve_G: not built yet");
}
