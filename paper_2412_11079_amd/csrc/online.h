// Internal declarations of the kernel-free pass (online.hip).
#pragma once

#include "uot_common.h"

namespace uot {

struct OnlineLaunch {
    PassLaunch P;             // strip, scalings, partials, stopping test (K, ldk unused)
    const double* y;          // m x dim target points
    const double* rows;       // n x 4: x'_i (2 c x_i, zero-padded to 3) and alpha_i = -c |x_i|^2
    const double* beta;       // m: beta_j = -c |y_j|^2
    const double* loga;       // n: log2 a_i (0 where a_i = 0)
    int32_t dim;              // 2 or 3
    // Column-tiled form (rows wider than one workgroup's columns): tile
    // blockIdx.y covers columns [t T, (t + 1) T), T = online_tile_cols().
    double* rowpart;          // tiles x n: the tiles' row sums (row pass)
    int32_t tiles;
};

// Rows of at most online_max_m() columns.
int64_t online_max_m();
// Rows a workgroup of the pass takes per group (and barrier).
int online_rows_per_group(int dim, int64_t m);
// Workgroups of the pass for rows of m columns that one compute unit holds.
int online_wgs_per_cu(int dim, int64_t m);
// Row and column terms of the exponent (rows, beta above) from the points
// and log2 a,
// c = cost_scale log2(e) / eps; once per solve.
hipError_t launch_online_setup(const double* x, const double* y, const double* a, int64_t n, int64_t m, int dim,
                               double c, double* rows, double* beta, double* loga, hipStream_t stream);
// One pass; mode MODE_FUSED or MODE_MARG.
hipError_t launch_online(int mode, const OnlineLaunch& O, hipStream_t stream);

// Column-tiled form for m > online_max_m(): per iteration a row pass (each
// tile's row sums of K v into rowpart), the row finish (tile sums in order;
// u, or with marginal != 0 the totals K v into P.s_out), then a column pass
// (column partials of K^T u per strip, summed by the column finalize).
// Grid: P.grid strips x tiles.
int64_t online_tile_cols();
int online_tile_wgs_per_cu(int dim);
hipError_t launch_online_tile_rows(const OnlineLaunch& O, hipStream_t stream);
hipError_t launch_online_row_finish(const OnlineLaunch& O, int marginal, hipStream_t stream);
hipError_t launch_online_tile_cols(const OnlineLaunch& O, hipStream_t stream);

}  // namespace uot
