// Library-internal entry points shared between the host sources.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "lem.h"

namespace lem {

class Arena;

// Records msg as the thread's last error and returns s.
lem_status set_error(lem_status s, const char* msg);

// y = exp(t A) x (+ phi_1(t A)(t g)) by the global method: a plan with
// LEM_METHOD_GLOBAL (calibration, then one step) whose device memory comes
// from `arena` when given (no hipMalloc/hipFree), else from hipMalloc.
// Synchronous; maps device-side failures to LEM_ERR_NOT_CONVERGED /
// LEM_ERR_NONFINITE.
lem_status global_expmv_in(const lem_operator* op, double t, const double* x, double* y,
                           int32_t n_states, double tol, int32_t m_max, void* stream,
                           Arena* arena);

// Upper bound on the device bytes global_expmv_in takes from an arena for
// this operator, ensemble size and Krylov limit (op must be non-NULL).
size_t global_expmv_bound(const lem_operator* op, int32_t n_states, int32_t m_max);

}  // namespace lem
