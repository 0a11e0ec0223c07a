// The DC-GK projected problem with lambda from the discrepancy principle.
#pragma once

#include "internal.h"

namespace dctk {

// lambda with ||beta_1 e_1 - C~_k y_lambda|| = target (the residual norm of
// the Krylov approximation), on the device, then y_lambda into st->y;
// k_use > 0 projects at min(k_use, steps).
hipError_t launch_projected_disc(dctk_ctx ctx, KState* st, double target, int k_use = 0);

}  // namespace dctk
