// Entry points whose implementation lands in later files; each returns an
// explicit error until then.
#include "ms_internal.h"

namespace ms {
ms_status warm_start(ms_ctx* c, double, int32_t*) { return fail(c, MS_E_ORDER, "warm start not available"); }
ms_status record_coarse(ms_ctx*) { return MS_OK; }
}  // namespace ms

extern "C" {
ms_status ms_set_warmstart(ms_ctx*, const ms_mlp_desc*) { return MS_E_ORDER; }
}
