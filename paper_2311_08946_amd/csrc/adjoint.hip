// Adjoint of the floating-row assembly with respect to the node samples.
#include <hip/hip_runtime.h>

#include "runtime.h"

using namespace pdd;

extern "C" pdd_status pdd_assemble_G_backward(pdd_system sys, const double* u, const double* lambda,
                                              double* g_axx, double* g_axy, double* g_ayy,
                                              double* g_bx, double* g_by, double* g_c, double* g_f,
                                              void* stream) {
  (void)sys; (void)u; (void)lambda; (void)g_axx; (void)g_axy; (void)g_ayy; (void)g_bx; (void)g_by;
  (void)g_c; (void)g_f; (void)stream;
  return fail(PDD_EINVAL, "pdd_assemble_G_backward: not built yet");
}
