// Internal declarations of the dense plan launchers (aux.hip).
#pragma once

#include "uot_common.h"

namespace uot {

// P_ij = s u_i (k_scale K_ij) v_j with s = *dscale (a device scalar) or 1.
hipError_t launch_plan_from_k(const void* K, int k_dtype, int64_t ldk, int64_t n, int64_t m, double k_scale,
                              const double* u, const double* v, void* P, int plan_dtype, int64_t ldp,
                              hipStream_t stream, const double* dscale = nullptr);
hipError_t launch_plan_from_cost(const double* C, int64_t ldc, int64_t n, int64_t m, double eps, const double* f,
                                 const double* g, void* P, int plan_dtype, int64_t ldp, hipStream_t stream);

}  // namespace uot
