// Internal declarations of the log-domain (log-sum-exp) pass (lse.hip).
#pragma once

#include "uot_common.h"

namespace uot {

// Potentials are kept in cost units (f = eps log u, g = eps log v); a pass at
// eps works in log2 units, F2 = c f, G2 = c g with c = log2(e) / eps.
struct LseLaunch {
    PassLaunch P;             // strip (rows_per_wg, grid, n, m), stopping test, flags (K, v, a, u unused)
    const void* C;            // n x ldc cost, FP64 or FP32 (c_dtype)
    int32_t c_dtype;          // UOT_F64 or UOT_F32
    int64_t ldc;
    double c;                 // log2(e) / eps of this pass
    double inv_c;             // eps ln 2 (potential = inv_c times its log2-unit value)
    double fi;                // tau / (tau + eps) of this pass
    const double* g;          // m column potentials (cost units)
    double* f;                // n row potentials (FUSED: written; MARG: read)
    const double* la2;        // n: log2 a_i (-inf where a_i = 0)
    double* r_out;            // MARG: row marginal r_i
    double* pmax;             // grid x ldp: per-workgroup column shifts (log2 units)
    float* psum;              // grid x ldp: per-workgroup column sums under those shifts
    int64_t ldp;
};

struct LseFinLaunch {
    const double* pmax;
    const float* psum;
    int64_t ldp;
    int32_t G;
    int64_t m;
    double c, inv_c, fi;
    const double* lb2;        // m: log2 b_j (-inf where b_j = 0)
    double* g;                // m column potentials (FUSED: updated; MARG: read)
    double* cprev;            // m: last column marginal (stopping test)
    double* c_out;            // MARG: column marginal
    Ctrl* ctrl;
    double* blockpart;        // 2 x blocks: sum |c - c_prev|, sum |c|
    int32_t marginal_only;
};

int64_t lse_max_m(int c_dtype);
// Workgroups of the pass that one compute unit holds (rows of m columns).
int lse_wgs_per_cu(int c_dtype, int64_t m);
// Per-solve setup: log2 a, log2 b.
hipError_t launch_lse_setup(const double* a, int64_t n, const double* b, int64_t m, double* la2, double* lb2,
                            hipStream_t stream);
// One pass (MODE_FUSED or MODE_MARG).
hipError_t launch_lse(int mode, const LseLaunch& L, hipStream_t stream);
// Column merge of the per-workgroup (shift, sum) pairs: new g, column
// marginal, stopping sums (FUSED) or the marginal alone (MARG).
hipError_t launch_lse_finalize(const LseFinLaunch& F, hipStream_t stream);
int lse_finalize_blocks(int64_t m);
// Copies of FP64 rows into FP32 storage (the cost read by an FP32 pass).
hipError_t launch_cost_to_f32(const double* C, int64_t ldc, int64_t n, int64_t m, float* out, int64_t ldo,
                              hipStream_t stream);

}  // namespace uot
