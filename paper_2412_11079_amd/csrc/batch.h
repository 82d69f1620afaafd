// Internal declarations of the batched solver (batch.hip).
#pragma once

#include <stddef.h>

#include "uot_common.h"

namespace uot {

// ---------------------------------------------------------------------------
// Batched problems (batch.hip)
// ---------------------------------------------------------------------------
struct BatchDesc {            // one problem, device-resident, in queue order
    const void* K;
    int64_t ldk;
    int64_t n, m;
    const double* a;          // n
    const double* b;          // m
    double* u;                // n
    double* v;                // m
    double* r;                // n
    double* c;                // m (also the previous marginal of the stopping test)
    double* loss;             // scalar
    uot_info* info;
    double fi;
    double k_scale;
    double eps;
    double tau;
    int32_t fi_is_one;
    int32_t shape;            // batch tile shape
    int64_t index;            // position of the problem in the caller's array
};

// The Python binding reads the shape and index words of packed descriptors.
static_assert(sizeof(BatchDesc) == 144, "BatchDesc layout");
static_assert(offsetof(BatchDesc, fi_is_one) == 128 && offsetof(BatchDesc, shape) == 132 &&
                  offsetof(BatchDesc, index) == 136,
              "BatchDesc layout");

struct BatchLaunch {
    const BatchDesc* desc;
    int32_t count;
    int32_t max_iter;
    double tol;
    int32_t check_every;
    int32_t pad0;
    int64_t m_lds;            // doubles per LDS vector (v and column sums)
    uint32_t* next;           // queue head (reset before each launch)
    uint64_t* trace;          // optional: 2 x count wall-clock stamps (start, end)
};

int batch_shape_count();
int64_t batch_shape_max_m(int shape, int k_dtype);
int batch_shape_rows(int shape);
bool batch_shape_ok(int shape, int k_dtype);
size_t batch_lds_bytes(int64_t m_lds);
int batch_max_grid(int k_dtype, size_t lds);
hipError_t launch_batch(int k_dtype, const BatchLaunch& B, int grid, size_t lds, hipStream_t stream);

}  // namespace uot
