// Kernel-free ("online") fused pass for a squared-Euclidean cost of 2-D or
// 3-D points: the iteration of Section 2.1 (vector form, rows first) with
// the Gibbs kernel recomputed in registers instead of streamed from HBM.
// The O(nm) memory traffic the paper identifies as the barrier (Sections 1
// and 3) disappears; what remains is arithmetic, so the pass is bounded by
// the vector ALU (VALU), not by HBM.
//
// Entry (i, j), in log2 units with exact FP64 arithmetic:
//   t_ij = -C_ij log2(e) / eps = alpha_i + beta_j + sum_d x'_id y_jd,
//   alpha_i = -|x_i|^2 c,  beta_j = -|y_j|^2 c,  x'_i = 2 c x_i,  c = cost_scale log2(e) / eps,
// then K_ij = 2^t_ij = 2^k 2^f with k = rint(t_ij) and f = t_ij - k in
// [-1/2, 1/2] (exact in FP64): 2^f by the hardware exp2 on the FP32
// rounding of f (relative error ~1e-7, the size of an FP32 storage
// rounding of K), 2^k by ldexp.  An FP32 argument would not do: t reaches
// hundreds, and its rounding alone would move K by ~1e-5.
//
// Workgroup: WG lanes owning a strip of rows; lane l holds the columns
// j = l + WG c (c < CPL, m <= WG CPL) in registers: coordinates and beta
// in FP64 (beta in LDS for the widest rows), v and the column partials in
// FP32.  Rows are taken R at a time
// (column-outer, row-inner, so each column's data serves R independent
// exponent chains): the R rows' K values are formed and dotted with v, the
// R row totals are reduced over the wave (FP64) and met in one LDS exchange
// and barrier (fixed order), lanes 0..R-1 of every wave form the R scalings
// u_i = (a_i / total_i)^fi at once, and a lane broadcast hands them to
// every lane, which accumulates the R rows into its column partials.  The
// column finalize sums the partials as for a stored K.  Row terms (x'_i,
// alpha_i) are wave-uniform and read by scalar loads.
#include "online.h"
#include "strip.h"

namespace uot {

__global__ void online_setup_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                    const double* __restrict__ a, int64_t n, int64_t m, int dim, double c,
                                    double* __restrict__ rows, double* __restrict__ beta,
                                    double* __restrict__ loga) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const double ai = a[t];
        loga[t] = ai > 0.0 ? log2(ai) : 0.0;
        double xd[3] = {0.0, 0.0, 0.0}, nx = 0.0;
        for (int d = 0; d < dim; ++d) {
            xd[d] = x[t * dim + d];
            nx = fma(xd[d], xd[d], nx);
        }
        for (int d = 0; d < 3; ++d) rows[4 * t + d] = 2.0 * c * xd[d];
        rows[4 * t + 3] = -c * nx;
    } else if (t - n < m) {
        const int64_t j = t - n;
        double ny = 0.0;
        for (int d = 0; d < dim; ++d) ny = fma(y[j * dim + d], y[j * dim + d], ny);
        beta[j] = -c * ny;
    }
}

// u = (a / s)^fi = 2^(fi (log2 a - log2 s)) at the precision of the pass's
// own entries: log2 s = e + log2(mant), the mantissa's log2 split as
// log2(mh) + ml / (mh ln 2) with mh its FP32 rounding (hardware log2, error
// ~6e-8 absolute on [-1, 0)) and ml = mant - mh exact; the exponent is
// kept in FP64 and split into an integer and a fraction in [-1/2, 1/2]
// for the hardware exp2 (relative error ~1e-7), the integer applied by
// ldexp.  Special totals follow the plain formula (0 -> +inf, +inf -> 0).
__device__ __forceinline__ double online_scaling(double log2a, double s, double fi) {
    if (s != s) return s;
    if (s == 0.0) return INFINITY;
    if (s == INFINITY) return 0.0;
    int e = 0;
    const double mt = frexp(s, &e);                   // [1/2, 1)
    const float mh = (float)mt;
    const float ml = (float)(mt - (double)mh);
    const float l2m = __builtin_amdgcn_logf(mh) + ml * __builtin_amdgcn_rcpf(mh) * 1.44269504f;
    const double y = fi * (log2a - ((double)e + (double)l2m));
    const double k = __builtin_rint(y);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(y - k)), (int)fmax(fmin(k, 2100.0), -2100.0));
}

constexpr int kOnlineRowsMax = 512;    // strip rows whose row inputs are staged in LDS (longer strips read HBM)

// BL: beta and v of the lane's columns sit in LDS (read once per group of R
// rows) instead of registers, for 16 columns per lane.
template <int DIM, int WG, int CPL, int R, int MODE, bool BL>
__global__ __launch_bounds__(WG) void online_kernel(OnlineLaunch O, const double* __restrict__ rows,
                                                    const double* __restrict__ beta) {
    static_assert(MODE == MODE_FUSED || MODE == MODE_MARG, "online fused or marginal pass");
    static_assert(R >= 1 && R <= 64, "rows per group");
    constexpr int NW = WG / 64;
    const PassLaunch& L = O.P;
    __shared__ double red[2][R][NW];
    __shared__ uint32_t exit_sh;
    __shared__ double row_a[kOnlineRowsMax], row_la[kOnlineRowsMax];   // a and log2 a (FUSED) or u (MARG)
    extern __shared__ __align__(16) double on_lds[];    // BL: beta (WG CPL), then v (WG CPL, FP32)

    if (pass_exit(L, &exit_sh)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);
    const int64_t m = L.m;
    // The strip's row inputs, read once: a group's chain after its barrier
    // then waits on LDS, not on HBM.
    const bool rows_in_lds = nrows <= kOnlineRowsMax;
    if (rows_in_lds)
        for (int k = tid; k < nrows; k += WG) {
            if constexpr (MODE == MODE_MARG) {
                row_a[k] = L.u[r0 + k];
            } else {
                row_a[k] = L.a[r0 + k];
                row_la[k] = O.loga[r0 + k];
            }
        }

    // The lane's columns (columns past m: a copy of the last one, v = 0).
    double yc[CPL][DIM], bc[BL ? 1 : CPL];
    float vc[BL ? 1 : CPL], acc[CPL];
    double* bl = on_lds;
    float* vl = (float*)(on_lds + (BL ? WG * CPL : 0));
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int64_t j = (int64_t)c * WG + tid;
        const int64_t jj = j < m ? j : m - 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) yc[c][d] = O.y[jj * DIM + d];
        if constexpr (BL) {
            bl[c * WG + tid] = beta[jj];
            vl[c * WG + tid] = j < m ? (float)L.v[j] : 0.0f;
        } else {
            bc[c] = beta[jj];
            vc[c] = j < m ? (float)L.v[j] : 0.0f;
        }
        acc[c] = 0.0f;
    }

    int slot = 0;
    for (int k = 0; k < nrows; k += R) {
        const int nr = nrows - k < R ? nrows - k : R;
        // Row terms of the group (rows past the strip repeat its last row;
        // their scaling is 0, so they add nothing).
        double xr[R][DIM], al[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = r0 + k + (r < nr ? r : nr - 1);
#pragma unroll
            for (int d = 0; d < DIM; ++d) xr[r][d] = rows[4 * i + d];
            al[r] = rows[4 * i + 3];
        }
        float kv[R][CPL], s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = 0.0f;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            // Each lane reads only the LDS words it wrote: no barrier needed.
            const double bcc = BL ? bl[c * WG + tid] : bc[BL ? 0 : c];
            const float vcc = BL ? vl[c * WG + tid] : vc[BL ? 0 : c];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double t = al[r] + bcc;
#pragma unroll
                for (int d = 0; d < DIM; ++d) t = fma(xr[r][d], yc[c][d], t);
                const double kf = __builtin_rint(t);
                const float f = (float)(t - kf);
                const float e = __builtin_ldexpf(__builtin_amdgcn_exp2f(f), (int)fmax(kf, -1000.0));
                kv[r][c] = e;
                s[r] = fmaf(e, vcc, s[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double d = wave_sum_f64((double)s[r]);
            if (lane == 0) red[slot][r][wave] = d;
        }
        __syncthreads();
        // Lane r (< nr) of every wave: row total in a fixed order, then u.
        double uu = 0.0;
        if (lane < nr) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tot += red[slot][lane][w];
            const int64_t i = r0 + k + lane;
            if constexpr (MODE == MODE_MARG) {
                uu = rows_in_lds ? row_a[k + lane] : L.u[i];
                if (wave == 0) L.s_out[i] = tot;
            } else {
                const double ai = rows_in_lds ? row_a[k + lane] : L.a[i];
                const double l2a = rows_in_lds ? row_la[k + lane] : O.loga[i];
                uu = ai == 0.0 ? 0.0 : L.fi_is_one ? ai / tot : online_scaling(l2a, tot, L.fi);
                if (wave == 0) {
                    L.u[i] = uu;
                    if (ai > 0.0 && !(tot > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
                    if (!isfinite(uu)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
                }
            }
        }
        slot ^= 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float fr = (float)readlane_f64(uu, r);
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[c] = fmaf(kv[r][c], fr, acc[c]);
        }
    }
    float* P = (float*)L.partials + (int64_t)blockIdx.x * L.ldp;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int64_t j = (int64_t)c * WG + tid;
        if (j < m) __builtin_nontemporal_store(acc[c], &P[j]);
    }
}

// ---------------------------------------------------------------------------
// Column-tiled form: rows wider than one workgroup's 8192 columns.  A row's
// total needs every tile before its scaling exists, so the fused pass
// splits into a row pass and a column pass that each form K again (twice
// the arithmetic of the fused pass).  Workgroup (strip, tile): 512 lanes,
// lane l holding columns t T + l + 512 c (c < 16) of tile t, coordinates
// in registers, beta (and v) in LDS as in the widest fused shape.
// ---------------------------------------------------------------------------
constexpr int kTileWG = 512;
constexpr int kTileCPL = 16;
constexpr int64_t kTileCols = (int64_t)kTileWG * kTileCPL;
constexpr int kTileRows = 8;              // rows per group (no K values are kept between phases)

int64_t online_tile_cols() { return kTileCols; }

// The lane's columns of tile blockIdx.y: coordinates into yc, beta (and v
// with WITH_V) into LDS; columns past m copy the last column (v = 0).
template <int DIM, bool WITH_V>
__device__ __forceinline__ void tile_columns(const OnlineLaunch& O, const double* __restrict__ beta, int64_t m,
                                             double (&yc)[kTileCPL][DIM], double* bl, float* vl) {
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * kTileCols;
#pragma unroll
    for (int c = 0; c < kTileCPL; ++c) {
        const int64_t j = j0 + (int64_t)c * kTileWG + tid;
        const int64_t jj = j < m ? j : m - 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) yc[c][d] = O.y[jj * DIM + d];
        bl[c * kTileWG + tid] = beta[jj];
        if constexpr (WITH_V) vl[c * kTileWG + tid] = j < m ? (float)O.P.v[j] : 0.0f;
    }
}

// 2^t of entry (row terms xr, al; column c) as in the fused pass.
template <int DIM>
__device__ __forceinline__ float tile_entry(const double (&xr)[DIM], double al, double bcc,
                                            const double (&ycc)[DIM]) {
    double t = al + bcc;
#pragma unroll
    for (int d = 0; d < DIM; ++d) t = fma(xr[d], ycc[d], t);
    const double kf = __builtin_rint(t);
    const float f = (float)(t - kf);
    return __builtin_ldexpf(__builtin_amdgcn_exp2f(f), (int)fmax(kf, -1000.0));
}

// Row pass: each tile's FP32 lane dots of its rows with v, reduced over the
// workgroup in FP64 (fixed order) into rowpart[tile n + i].
template <int DIM>
__global__ __launch_bounds__(kTileWG) void online_tile_rows_kernel(OnlineLaunch O, const double* __restrict__ rows,
                                                                  const double* __restrict__ beta) {
    constexpr int NW = kTileWG / 64;
    constexpr int R = kTileRows;
    const PassLaunch& L = O.P;
    __shared__ double red[2][R][NW];
    __shared__ uint32_t exit_sh;
    extern __shared__ __align__(16) double on_lds[];    // beta (T), then v (T, FP32)
    if (pass_exit(L, &exit_sh)) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);
    double yc[kTileCPL][DIM];
    double* bl = on_lds;
    float* vl = (float*)(on_lds + kTileCols);
    tile_columns<DIM, true>(O, beta, L.m, yc, bl, vl);
    double* out = O.rowpart + (int64_t)blockIdx.y * L.n;
    int slot = 0;
    for (int k = 0; k < nrows; k += R) {
        const int nr = nrows - k < R ? nrows - k : R;
        double xr[R][DIM], al[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = r0 + k + (r < nr ? r : nr - 1);
#pragma unroll
            for (int d = 0; d < DIM; ++d) xr[r][d] = rows[4 * i + d];
            al[r] = rows[4 * i + 3];
        }
        float s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = 0.0f;
#pragma unroll
        for (int c = 0; c < kTileCPL; ++c) {
            // Each lane reads only the LDS words it wrote: no barrier needed.
            const double bcc = bl[c * kTileWG + tid];
            const float vcc = vl[c * kTileWG + tid];
#pragma unroll
            for (int r = 0; r < R; ++r) s[r] = fmaf(tile_entry<DIM>(xr[r], al[r], bcc, yc[c]), vcc, s[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double d = wave_sum_f64((double)s[r]);
            if (lane == 0) red[slot][r][wave] = d;
        }
        __syncthreads();
        if (wave == 0 && lane < nr) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tot += red[slot][lane][w];
            out[r0 + k + lane] = tot;
        }
        slot ^= 1;
    }
}

// Row finish: s_i = sum of the tiles' row sums in tile order; then u_i
// (fused step) or, with marginal, s_i itself into s_out.
__global__ void online_row_finish_kernel(OnlineLaunch O, int marginal) {
    const PassLaunch& L = O.P;
    if (!marginal && L.check_done && ld_volatile_u32(&L.ctrl->done) != 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    double tot = 0.0;
    for (int t = 0; t < O.tiles; ++t) tot += O.rowpart[(int64_t)t * L.n + i];
    if (marginal) {
        L.s_out[i] = tot;
        return;
    }
    const double ai = L.a[i];
    const double uu = ai == 0.0 ? 0.0 : L.fi_is_one ? ai / tot : online_scaling(O.loga[i], tot, L.fi);
    L.u[i] = uu;
    if (ai > 0.0 && !(tot > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
    if (!isfinite(uu)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
}

// Column pass: each tile's column partials of K^T u over its strip rows
// (u staged in LDS), no cross-lane exchange at all.
template <int DIM>
__global__ __launch_bounds__(kTileWG) void online_tile_cols_kernel(OnlineLaunch O, const double* __restrict__ rows,
                                                                  const double* __restrict__ beta) {
    constexpr int R = kTileRows;
    const PassLaunch& L = O.P;
    __shared__ uint32_t exit_sh;
    __shared__ double row_u[kOnlineRowsMax];
    extern __shared__ __align__(16) double on_lds[];    // beta (T)
    if (pass_exit(L, &exit_sh)) return;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);
    const int64_t m = L.m;
    const bool rows_in_lds = nrows <= kOnlineRowsMax;
    if (rows_in_lds)
        for (int k = tid; k < nrows; k += kTileWG) row_u[k] = L.u[r0 + k];
    double yc[kTileCPL][DIM];
    double* bl = on_lds;
    tile_columns<DIM, false>(O, beta, m, yc, bl, nullptr);
    float acc[kTileCPL];
#pragma unroll
    for (int c = 0; c < kTileCPL; ++c) acc[c] = 0.0f;
    __syncthreads();
    for (int k = 0; k < nrows; k += R) {
        const int nr = nrows - k < R ? nrows - k : R;
        double xr[R][DIM], al[R];
        float ur[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int rr = r < nr ? r : nr - 1;
            const int64_t i = r0 + k + rr;
#pragma unroll
            for (int d = 0; d < DIM; ++d) xr[r][d] = rows[4 * i + d];
            al[r] = rows[4 * i + 3];
            // rows past the strip repeat its last row with scaling 0
            ur[r] = r < nr ? (float)(rows_in_lds ? row_u[k + rr] : L.u[i]) : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < kTileCPL; ++c) {
            const double bcc = bl[c * kTileWG + tid];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[c] = fmaf(tile_entry<DIM>(xr[r], al[r], bcc, yc[c]), ur[r], acc[c]);
        }
    }
    float* P = (float*)L.partials + (int64_t)blockIdx.x * L.ldp;
    const int64_t j0 = (int64_t)blockIdx.y * kTileCols;
#pragma unroll
    for (int c = 0; c < kTileCPL; ++c) {
        const int64_t j = j0 + (int64_t)c * kTileWG + tid;
        if (j < m) __builtin_nontemporal_store(acc[c], &P[j]);
    }
}

static constexpr size_t kTileRowsLds = (size_t)kTileCols * 12;   // beta FP64 + v FP32
static constexpr size_t kTileColsLds = (size_t)kTileCols * 8;    // beta FP64

int online_tile_wgs_per_cu(int dim) {
    int nb = 0;
    hipError_t e = dim == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, online_tile_rows_kernel<2>, kTileWG,
                                                                           kTileRowsLds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, online_tile_rows_kernel<3>, kTileWG,
                                                                           kTileRowsLds);
    return e == hipSuccess ? nb : 0;
}

template <typename Fn>
static hipError_t tile_launch(Fn fn, size_t lds, const OnlineLaunch& O, hipStream_t stream) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(O.P.grid, O.tiles), dim3(kTileWG), lds, stream, O, O.rows, O.beta);
    return hipGetLastError();
}

hipError_t launch_online_tile_rows(const OnlineLaunch& O, hipStream_t stream) {
    if (O.dim == 2) return tile_launch(online_tile_rows_kernel<2>, kTileRowsLds, O, stream);
    if (O.dim == 3) return tile_launch(online_tile_rows_kernel<3>, kTileRowsLds, O, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_online_tile_cols(const OnlineLaunch& O, hipStream_t stream) {
    if (O.dim == 2) return tile_launch(online_tile_cols_kernel<2>, kTileColsLds, O, stream);
    if (O.dim == 3) return tile_launch(online_tile_cols_kernel<3>, kTileColsLds, O, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_online_row_finish(const OnlineLaunch& O, int marginal, hipStream_t stream) {
    const unsigned blocks = (unsigned)((O.P.n + 255) / 256);
    hipLaunchKernelGGL(online_row_finish_kernel, dim3(blocks), dim3(256), 0, stream, O, marginal);
    return hipGetLastError();
}

hipError_t launch_online_setup(const double* x, const double* y, const double* a, int64_t n, int64_t m, int dim,
                               double c, double* rows, double* beta, double* loga, hipStream_t stream) {
    const int64_t total = n + m;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(online_setup_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, y, a, n, m, dim, c,
                       rows, beta, loga);
    return hipGetLastError();
}

// Lanes per workgroup (WG), columns per lane (CPL) and rows per group (R)
// for rows of m columns: the R CPL K values of a group stay in registers
// until its scalings are known; BL puts beta and v in LDS.  At 16 columns
// per lane, 4 rows per group (3-D: a few values spilled, still faster than
// 3 rows; 2-D: 5 rows were slower).
#ifndef UOT_ONLINE_WIDE
#define UOT_ONLINE_WIDE(DIM, X) X(DIM, 512, 16, 4, true)
#endif
#define UOT_ONLINE_SHAPES(DIM, X)                   \
    if (m <= 512) X(DIM, 512, 1, 8, false);         \
    else if (m <= 1024) X(DIM, 512, 2, 8, false);   \
    else if (m <= 2048) X(DIM, 512, 4, 8, false);   \
    else if (m <= 4096) X(DIM, 512, 8, 8, false);   \
    else UOT_ONLINE_WIDE(DIM, X)

// Dynamic LDS of a shape: beta (FP64) and v (FP32) of every column with BL.
static constexpr size_t online_lds_of(int wg, int cpl, bool bl) { return bl ? (size_t)wg * cpl * 12 : 0; }

int64_t online_max_m() { return 8192; }

int online_rows_per_group(int dim, int64_t m) {
    int rg = 0;
#define UOT_RG(DIM, WG, CPL, R, BL) rg = R
    if (dim == 2) {
        UOT_ONLINE_SHAPES(2, UOT_RG);
    } else {
        UOT_ONLINE_SHAPES(3, UOT_RG);
    }
#undef UOT_RG
    return rg;
}

int online_wgs_per_cu(int dim, int64_t m) {
    int nb = 0;
    hipError_t e = hipSuccess;
#define UOT_OCC(DIM, WG, CPL, R, BL)                                                                          \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, online_kernel<DIM, WG, CPL, R, MODE_FUSED, BL>, WG, \
                                                     online_lds_of(WG, CPL, BL))
    if (dim == 2) {
        UOT_ONLINE_SHAPES(2, UOT_OCC);
    } else {
        UOT_ONLINE_SHAPES(3, UOT_OCC);
    }
#undef UOT_OCC
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_online(int mode, const OnlineLaunch& O, hipStream_t stream) {
    const int64_t m = O.P.m;
    if ((O.dim != 2 && O.dim != 3) || m > online_max_m() || (mode != MODE_FUSED && mode != MODE_MARG))
        return hipErrorInvalidValue;
#define UOT_LAUNCH(DIM, WG, CPL, R, BL)                                                                         \
    do {                                                                                                        \
        auto kf = online_kernel<DIM, WG, CPL, R, MODE_FUSED, BL>;                                               \
        auto km = online_kernel<DIM, WG, CPL, R, MODE_MARG, BL>;                                                \
        auto kk = mode == MODE_FUSED ? kf : km;                                                                 \
        const size_t lds = online_lds_of(WG, CPL, BL);                                                          \
        if (lds > 65536) {                                                                                      \
            hipError_t ea = hipFuncSetAttribute((const void*)kk, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                                (int)lds);                                                      \
            if (ea != hipSuccess) return ea;                                                                    \
        }                                                                                                       \
        hipLaunchKernelGGL(kk, dim3(O.P.grid), dim3(WG), lds, stream, O, O.rows, O.beta);                      \
    } while (0)
    if (O.dim == 2) {
        UOT_ONLINE_SHAPES(2, UOT_LAUNCH);
    } else {
        UOT_ONLINE_SHAPES(3, UOT_LAUNCH);
    }
#undef UOT_LAUNCH
    return hipGetLastError();
}

}  // namespace uot
