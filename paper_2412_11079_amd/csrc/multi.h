// Internal declarations of the multi-right-hand-side solver (multi.hip).
#pragma once

#include "uot_common.h"

namespace uot {

// Out^T[r][i] = sum_k A[i][k] X^T[r][k]: A (rows x kdim, row-major, lda)
// times R right-hand sides held k-contiguous (X^T, R_pad x ldx), split over
// kdim into `splits` chunks; chunk s's FP32 sum for (r, i) goes to
// part[mpart_index(r, i, s, ld_part, splits)] (splits x R_pad x ld_part
// floats in all).
// Partial-sum layout: for each right-hand side r and block of 32 rows i,
// the splits' 32 sums follow one another (128 bytes each), so a GEMM
// workgroup stores whole 128-byte runs and the epilogue reads all chunks of
// 32 rows as one contiguous run.  ld_part is a multiple of 32.
__host__ __device__ inline int64_t mpart_index(int64_t r, int64_t i, int s, int64_t ld_part, int splits) {
    return ((r * (ld_part >> 5) + (i >> 5)) * splits + s) * 32 + (i & 31);
}

struct MGemm {
    const void* A;
    int64_t lda;
    int64_t rows;        // valid rows of A (rows beyond read 0)
    int64_t rows_pad;    // multiple of the row tile
    int64_t kdim_pad;    // multiple of the k step; A columns and X entries beyond kdim must be finite / 0
    const void* x_hi;    // BF16 form: high parts; FP32 form: the values
    const void* x_lo;    // BF16 form: low parts (x - hi, rounded)
    int64_t ldx;         // elements between consecutive right-hand sides
    int64_t r_pad;       // multiple of the column tile
    int32_t splits;
    int64_t kchunk;      // multiple of the k step
    float* part;
    int64_t ld_part;     // = rows_pad
    int32_t blocked;     // ring variants: A is in the tiled layout of launch_mpack (lda unused)
    int32_t variant;     // 0: fragments loaded by each wave; 1: 128 x 128 tiles staged through LDS;
                         // BF16 only, A in the tiled layout of launch_mpack, tiles through LDS
                         // with a ring of loads in flight: 3: 256 x 256, 4: 128 x 128
};

// After a GEMM: S[r][i] = sum_s part[s][r][i] (FP64, fixed order), then
//   mode 0 (update):   y = (T / (k_scale S))^fi, written to y_out (FP64,
//                      R x ld_y) and as the next GEMM's right-hand sides
//                      (BF16 hi/lo or FP32, R_pad x ld_next, zero padding);
//                      optionally marg = y * k_scale S;
//   mode 1 (marginal): marg = y_in * k_scale S.
struct MEpi {
    const float* part;
    int64_t ld_part;
    int32_t splits;
    int64_t rows;        // valid rows (n or m)
    int64_t R;
    int64_t r_pad;
    const double* target;   // R x rows (histograms as rows)
    double* y;              // R x rows (scalings out, or in for mode 1)
    double* marg;           // R x rows, optional
    void* next_hi;          // R_pad x ld_next (mode 0)
    void* next_lo;
    int64_t ld_next;        // >= rows, multiple of 64
    int32_t bf16;           // next right-hand sides as BF16 hi/lo (1) or FP32 (0)
    double fi;
    int32_t fi_is_one;
    double k_scale;
    int32_t mode;
    int32_t store_y;        // mode 0: also write y (the final iteration's scalings)
    uint32_t* flags;
};

hipError_t launch_mgemm(int bf16, const MGemm& G, hipStream_t stream);
hipError_t launch_mepi(const MEpi& E, hipStream_t stream);
// KT (m x ldkt) = K^T for a stored K (n x ldk), padding columns of KT zero.
hipError_t launch_transpose(int k_dtype, const void* K, int64_t ldk, int64_t n, int64_t m, void* KT, int64_t ldkt,
                            hipStream_t stream);
// BF16 A operand in the tiled layout read by the ring products: block
// (rb, kb) holds rows 256 rb .. 256 rb + 255 and k values 32 kb .. 32 kb + 31
// as 256 rows of 64 bytes (16 KiB, contiguous), blocks running along k
// first, so one stage of a workgroup's tile is one contiguous read.
// dst (rows_pad x kdim_pad, both multiples of 256 and 32) gets
// A[row][k] = trans ? src[k][row] : src[row][k] where the source entry
// exists (src: src_rows x src_cols, leading dimension ld), else 0.
hipError_t launch_mpack(int trans, const void* src, int64_t ld, int64_t src_rows, int64_t src_cols, void* dst,
                        int64_t rows_pad, int64_t kdim_pad, hipStream_t stream);
constexpr int64_t kMPackRows = 256;
constexpr int64_t kMPackK = 32;

// Right-hand sides of the first iteration: v = 1 for r < R, j < m, else 0.
hipError_t launch_ones_rhs(int bf16, void* hi, void* lo, int64_t R, int64_t r_pad, int64_t m, int64_t ld,
                           hipStream_t stream);
// Per right-hand side objective (one workgroup per r) from u, v, r, c, a, b.
hipError_t launch_multi_loss(const double* U, const double* V, const double* Rm, const double* Cm, const double* A,
                             const double* B, int64_t n, int64_t m, int64_t R, double eps, double tau, int fi_is_one,
                             double* losses, uint32_t* flags, hipStream_t stream);

// reset != 0: clear *flags; else write info (iters, flags).
hipError_t launch_multi_info(uot_info* info, int64_t iters, uint32_t* flags, int reset, hipStream_t stream);

constexpr int kMTileRows = 128;   // rows of A per workgroup
constexpr int kMTileCols = 128;   // right-hand sides per workgroup
constexpr int kMStep = 16;        // k per step (BF16); the FP32 form steps by 8
constexpr int kMBigRows = 256;    // BF16 256 x 256 variant: rows of A per workgroup
constexpr int kMBigCols = 256;    // and right-hand sides per workgroup

}  // namespace uot
