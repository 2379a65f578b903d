// Space-time interpolation-based FMM (placeholder until the far field lands).
#include "ifmm.h"

namespace tdbem {
void ifmm_setup(tdbem_ctx *) { throw Error{TDBEM_EINVAL, "IFMM mode is not built yet"}; }
void ifmm_reset(tdbem_ctx *) {}
void ifmm_destroy(tdbem_ctx *) {}
void ifmm_subtract_far(tdbem_ctx *, int, double *, hipStream_t) {}
void ifmm_add_far(tdbem_ctx *, int, double *, hipStream_t) {}
void ifmm_after_solve(tdbem_ctx *, int, hipStream_t) {}
}  // namespace tdbem
