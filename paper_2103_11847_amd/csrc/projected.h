// DC-GK projected problems beyond GCV: lambda from the discrepancy
// principle, the stopping index from the L-curve.
#pragma once

#include "internal.h"

namespace dctk {

// lambda with ||beta_1 e_1 - C~_k y_lambda|| = target (the residual norm of
// the Krylov approximation), on the device, then y_lambda into st->y;
// k_use > 0 projects at min(k_use, steps).
hipError_t launch_projected_disc(dctk_ctx ctx, KState* st, double target, int k_use = 0);

// The L-curve corner of the LSQR stopping index over the steps taken: y of
// the corner's LSQR iterate into st->y (zero beyond it), the index into
// st->sweeps, its residual norm into st->resnorm.
hipError_t launch_lcurve(dctk_ctx ctx, KState* st);

}  // namespace dctk
