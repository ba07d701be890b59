// Entry points whose implementation lands in later files; each returns an
// explicit error until then.
#include "ms_internal.h"

namespace ms {
void launch_coarse_correction(ms_ctx*, int) {}
ms_status launch_galerkin(ms_ctx* c, int) { return fail(c, MS_E_ORDER, "two-level preconditioner not available"); }
ms_status coarse_factor(ms_ctx* c) { return fail(c, MS_E_ORDER, "two-level preconditioner not available"); }
ms_status paper_step(ms_ctx* c, double, const ms_solver_params&, ms_step_stats*) {
  return fail(c, MS_E_ORDER, "paper mode not available");
}
ms_status warm_start(ms_ctx* c, double, int32_t*) { return fail(c, MS_E_ORDER, "warm start not available"); }
ms_status record_coarse(ms_ctx*) { return MS_OK; }
}  // namespace ms

extern "C" {
ms_status ms_build_basis(ms_ctx* c, const ms_basis_params*) { return ms::fail(c, MS_E_ORDER, "not available"); }
ms_status ms_set_basis(ms_ctx* c, int32_t, const double*, const int64_t*, const int32_t*, const double*) {
  return ms::fail(c, MS_E_ORDER, "not available");
}
ms_status ms_get_basis_size(const ms_ctx*, int32_t*, int64_t*) { return MS_E_ORDER; }
ms_status ms_get_basis(const ms_ctx*, double*, int64_t*, int32_t*, double*, int32_t*) { return MS_E_ORDER; }
ms_status ms_get_coarse(ms_ctx*, double*) { return MS_E_ORDER; }
ms_status ms_set_warmstart(ms_ctx*, const ms_mlp_desc*) { return MS_E_ORDER; }
ms_status ms_get_coarse_matrix(ms_ctx*, double*) { return MS_E_ORDER; }
ms_status ms_batch_step(ms_ctx* const*, int32_t, double, const ms_solver_params*, ms_step_stats*) {
  return MS_E_ORDER;
}
}
