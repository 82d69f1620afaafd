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
    // A large problem may be split by rows into `parts` queue entries (part
    // `part` holds the rows that K, a, u, r point at here; n is its row
    // count; b, v, c and the other outputs are the problem's).  The parts
    // exchange their column sums once per iteration through the exchange
    // pool: header `split` (a counter and a flag word) and the area `xch`
    // bytes from the pool's start (see batch.hip).
    int32_t part;
    int32_t parts;
    int32_t split;
    int32_t pad0;
    int64_t xch;
    int64_t pad1;
};

// The Python binding reads the shape and index words of packed descriptors.
static_assert(sizeof(BatchDesc) == 176, "BatchDesc layout");
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
    unsigned char* pool;      // exchange pool of split problems (headers first)
    int32_t nsplit;           // split problems (headers to clear before the launch)
    int32_t pad1;
};

// Exchange pool: nsplit headers of kBatchHeaderBytes (a uint32 counter and a
// uint32 flag word, cleared before each launch), then one area per split
// problem of P parts over m columns (FP64 words, mx = m rounded up to even):
// column sums 2 x P x mx (by iteration parity), each part's column marginal
// P x mx, the parts' objective row terms P x 4.
inline size_t batch_xch_bytes(int parts, int64_t m) {
    const int64_t mx = (m + 1) / 2 * 2;
    return sizeof(double) * ((size_t)3 * parts * mx + (size_t)4 * parts);
}
constexpr size_t kBatchHeaderBytes = 16;   // per split problem: counter, flags

int batch_shape_count();
int64_t batch_shape_max_m(int shape, int k_dtype);
int batch_shape_rows(int shape);
int batch_shape_chunks(int shape);
bool batch_shape_ok(int shape, int k_dtype);
size_t batch_lds_bytes(int64_t m_lds);
int batch_max_grid(int k_dtype, size_t lds);
hipError_t launch_batch(int k_dtype, const BatchLaunch& B, int grid, size_t lds, hipStream_t stream);

}  // namespace uot
