// Far-field (IFMM) hooks of the marching driver.
#pragma once
#include "tdbem_internal.h"

namespace tdbem {
void ifmm_setup(tdbem_ctx *C);                                   // tables, lists, operators, state
void ifmm_reset(tdbem_ctx *C);                                   // zero all far-field state
void ifmm_destroy(tdbem_ctx *C);
// rhs[e][r] -= far-field potential deposited for step alpha (target slot alpha-1)
void ifmm_subtract_far(tdbem_ctx *C, int alpha, double *rhs, hipStream_t s);
const double *ifmm_far_slot(const tdbem_ctx *C, int alpha);
// out[e][r] += far-field potential deposited for step alpha
void ifmm_add_far(tdbem_ctx *C, int alpha, double *out, hipStream_t s);
// after J^{alpha-1} is in the history ring: upward/downward passes at time gates
void ifmm_after_solve(tdbem_ctx *C, int alpha, hipStream_t s);
// marching state of the far field (moments, local expansions, pending L2L
// contributions, far-field ring): its size in bytes, and a copy to (save) or
// from host memory, stream-ordered on s
size_t ifmm_state_bytes(const tdbem_ctx *C);
void ifmm_state_copy(tdbem_ctx *C, char *host, bool save, hipStream_t s);
}  // namespace tdbem
