// Log-domain (log-sum-exp) fused pass: the iteration of Section 2.1 on the
// potentials f = eps log u, g = eps log v,
//     f_i = fi (eps log a_i - eps LSE_j((g_j - C_ij)/eps))
//     g_j = fi (eps log b_j - eps LSE_i((f_i - C_ij)/eps)),
// reading the stored cost C (FP64, or FP32) once per iteration.  No
// exponential exceeds 1 (every sum is taken under its maximum), so the pass
// runs at any eps without absorption; in log2 units (c = log2(e)/eps) an
// entry's row term is 2^(G2_j - c C_ij - M_i) and its column term
// 2^(F2_i - c C_ij - S_j).
//
// Workgroup: 512 lanes over a strip of rows, a row streamed through 16-byte
// chunks (NC per lane, up to 16 entries, two rows in flight) as in the
// stored-kernel pass.  Per row: (1) each lane forms its entries' exponents
// in FP64 and their maximum, (2) the sum of 2^(z - lane max) in FP32, (3)
// the lanes' (max, sum) pairs are merged over the wave and then the waves'
// pairs over 8 lanes through LDS, in a fixed order (FP64), giving the row
// LSE and the new F2_i, and (4) each lane adds the row's column terms to
// its columns' running sums.  A column's running shift is raised (with a
// margin of 32 in log2 units, so it rarely moves) when a term would exceed
// it, rescaling the sum; one wave-wide test per row decides whether any
// lane must.  The column finalize merges the workgroups' (shift, sum) pairs.
#include "lse.h"
#include "scalemath.h"
#include "strip.h"

namespace uot {

constexpr int kLseWG = 512;
constexpr int kLseRowsMax = 1024;      // strip rows whose row inputs are staged in LDS (longer strips read HBM)
constexpr double kColMargin = 32.0;    // log2 headroom of a raised column shift
constexpr double kLog2E = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// log2 of a finite s > 0, and 2^x for any x.
__device__ __forceinline__ double log2_pos(double s) { return sm::log_pos(s) * kLog2E; }
__device__ __forceinline__ double exp2_any(double x) { return sm::exp_any(x * kLn2); }

template <typename CT>
__device__ __forceinline__ double cost_at(const u32x4& w, int e);
template <>
__device__ __forceinline__ double cost_at<double>(const u32x4& w, int e) {
    return __hiloint2double((int)w[2 * e + 1], (int)w[2 * e]);
}
template <>
__device__ __forceinline__ double cost_at<float>(const u32x4& w, int e) {
    return (double)__int_as_float((int)w[e]);
}

// Maximum over the 64 lanes of a wave (exact, so every lane gets the same
// value whatever the exchange pattern): the row-of-16 butterfly of
// wave_sum_f64 with fmax, then the four rows through readlane.
__device__ __forceinline__ double wave_max_dpp(double x) {
    x = fmax(x, dpp_f64<0xB1>(x));     // quad_perm [1,0,3,2]
    x = fmax(x, dpp_f64<0x4E>(x));     // quad_perm [2,3,0,1]
    x = fmax(x, dpp_f64<0x141>(x));    // row_half_mirror
    x = fmax(x, dpp_f64<0x140>(x));    // row_mirror
    return fmax(fmax(readlane_f64(x, 0), readlane_f64(x, 16)), fmax(readlane_f64(x, 32), readlane_f64(x, 48)));
}

// Maximum over aligned groups of 8 lanes (lanes 0-7 of a row of 16 hold the
// waves' values).
__device__ __forceinline__ double group8_max(double x) {
    x = fmax(x, dpp_f64<0xB1>(x));
    x = fmax(x, dpp_f64<0x4E>(x));
    x = fmax(x, dpp_f64<0x141>(x));
    return x;
}

template <typename CT, int WG, int NC, int D, int MODE>
__global__ __launch_bounds__(WG) void lse_kernel(LseLaunch L) {
    static_assert(MODE == MODE_FUSED || MODE == MODE_MARG, "fused or marginal pass");
    constexpr int NW = WG / 64;
    static_assert(NW <= 8, "the waves' row pairs are merged in one group of 8 lanes");
    constexpr int V = 16 / (int)sizeof(CT);
    constexpr int E = NC * V;
    const PassLaunch& P = L.P;
    __shared__ double red[2][2][NW];
    __shared__ uint32_t exit_sh;
    __shared__ double rowv[kLseRowsMax];       // the strip's log2 a_i (FUSED) or f_i (MARG)
    extern __shared__ __align__(16) double g2s[];     // G2 of every column

    if (pass_exit(P, &exit_sh)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t m = P.m;
    const int64_t r0 = (int64_t)blockIdx.x * P.rows_per_wg;
    int64_t r1 = r0 + P.rows_per_wg;
    if (r1 > P.n) r1 = P.n;
    const int nrows = (int)(r1 - r0);
    const double c = L.c;

    // G2 of every column the lanes cover (E per lane): -inf past m, so those
    // entries add nothing to the row sums.
    for (int j = tid; j < WG * E; j += WG) g2s[j] = j < m ? c * L.g[j] : -INFINITY;
    // The strip's row inputs (log2 a, or f for the marginal pass), read once:
    // the row's chain after its barrier then waits on LDS, not on an HBM load.
    const bool in_lds = nrows <= kLseRowsMax;
    if (in_lds)
        for (int k = tid; k < nrows; k += WG) rowv[k] = MODE == MODE_MARG ? L.f[r0 + k] : L.la2[r0 + k];

    // Buffer resource over the strip: chunks of lanes past column m and rows
    // past the strip read 0 (they are masked below).
    const uint32_t row_bytes = (uint32_t)(L.ldc * (int64_t)sizeof(CT));
    const uint32_t strip_bytes = (uint32_t)nrows * row_bytes;
    const CT* strip = (const CT*)L.C + r0 * L.ldc;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)strip, (short)0, (int)strip_bytes, kBufferWord3);
    int64_t col[NC];
    uint32_t voff[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        col[q] = ((int64_t)(wave * NC + q) * 64 + lane) * V;
        voff[q] = col[q] < m ? (uint32_t)(col[q] * (int64_t)sizeof(CT)) : strip_bytes;
    }
    // Entry x = q V + e is column col[q] + e (< WG E: its LDS word exists);
    // columns past m read cost 0 and G2 = -inf, and their running column sums
    // (never stored) take no part in the shift test.
    int jc[E];
    bool ok[E];
    double cm[E];
    float cs[E];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int64_t j = col[q] + e;
            ok[q * V + e] = j < m;
            jc[q * V + e] = (int)j;
        }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        cm[e] = -1e300;
        cs[e] = 0.0f;
    }
    u32x4 buf[D][NC];
    auto load = [&](int bq, int k) {
        const uint32_t soff = (uint32_t)k * row_bytes;
#pragma unroll
        for (int q = 0; q < NC; ++q)
            buf[bq][q] = __builtin_bit_cast(
                u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(voff[q] + soff), 0, kLoadAux));
    };
#pragma unroll
    for (int q = 0; q < D - 1; ++q) load(q, q);
    __syncthreads();

    int slot = 0;
    for (int k0 = 0; k0 < nrows; k0 += D) {
#pragma unroll
        for (int bq = 0; bq < D; ++bq) {
            const int k = k0 + bq;
            if (k >= nrows) continue;
            load((bq + D - 1) % D, k + D - 1);
            const int64_t i = r0 + k;
            // (1) exponents G2_j - c C_ij (FP64) and their lane maximum,
            // (2) the lane sum under that maximum
            double z[E];
            double ml = -1e300;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    z[q * V + e] = fma(-cost_at<CT>(buf[bq][q], e), c, g2s[jc[q * V + e]]);
                    ml = fmax(ml, z[q * V + e]);
                }
            float sl = 0.0f;
#pragma unroll
            for (int x = 0; x < E; ++x) sl += __builtin_amdgcn_exp2f((float)(z[x] - ml));
            // (3) merge over the wave, then the waves' pairs in lanes 0..NW-1
            // of every wave (fixed order: the same bits everywhere)
            const double mw = wave_max_dpp(ml);
            const double sw = wave_sum_f64((double)(sl * __builtin_amdgcn_exp2f((float)(ml - mw))));
            if (lane == 0) {
                red[slot][0][wave] = mw;
                red[slot][1][wave] = sw;
            }
            __syncthreads();
            const int gl = lane & 7;
            const double mg = gl < NW ? red[slot][0][gl] : -1e300;
            const double M = readlane_f64(group8_max(mg), 0);
            const double sg = gl < NW ? red[slot][1][gl] * (double)__builtin_amdgcn_exp2f((float)(mg - M)) : 0.0;
            const double S = readlane_f64(group_sum_f64<8>(sg), 0);
            slot ^= 1;
            const double lse2 = S > 0.0 ? M + log2_pos(S) : -INFINITY;     // log2 sum_j 2^(G2_j - c C_ij)
            double F2;
            if constexpr (MODE == MODE_MARG) {
                F2 = c * (in_lds ? rowv[k] : L.f[i]);
                if (tid == 0) L.r_out[i] = F2 == -INFINITY ? 0.0 : exp2_any(F2 + lse2);
            } else {
                const double la = in_lds ? rowv[k] : L.la2[i];
                F2 = la == -INFINITY ? -INFINITY : L.fi * (la - lse2);
                if (tid == 0) {
                    L.f[i] = F2 * L.inv_c;
                    if (la != -INFINITY && !(S > 0.0)) atomicOr(&P.ctrl->flags, UOT_FLAG_ZERO_SUM);
                    if (la != -INFINITY && !isfinite(F2)) atomicOr(&P.ctrl->flags, UOT_FLAG_NONFINITE);
                }
            }
            // (4) column terms 2^(F2 - c C_ij) into the running sums; a shift
            // is raised only where a term exceeds it (one wave-wide test)
            bool raise = false;
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int x = q * V + e;
                    z[x] = fma(-cost_at<CT>(buf[bq][q], e), c, F2);
                    raise |= ok[x] && z[x] > cm[x];
                }
            if (__builtin_amdgcn_ballot_w64(raise) != 0) {
#pragma unroll
                for (int x = 0; x < E; ++x)
                    if (ok[x] && z[x] > cm[x]) {
                        const double nm = z[x] + kColMargin;
                        cs[x] *= __builtin_amdgcn_exp2f((float)(cm[x] - nm));
                        cm[x] = nm;
                    }
            }
#pragma unroll
            for (int x = 0; x < E; ++x) cs[x] += __builtin_amdgcn_exp2f((float)(z[x] - cm[x]));
        }
    }
    double* pm = L.pmax + (int64_t)blockIdx.x * L.ldp;
    float* ps = L.psum + (int64_t)blockIdx.x * L.ldp;
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (col[q] + e < m) {
                pm[col[q] + e] = cm[q * V + e];
                ps[col[q] + e] = cs[q * V + e];
            }
}

// Column merge: a block of 256 threads takes 32 columns; thread (col, ph)
// with col = tid % 32 and phase ph = tid / 32 covers workgroups ph, ph + 8,
// ...  The phases' maxima and then their sums under the common maximum are
// combined through LDS in phase order, so the result does not depend on
// timing.
constexpr int kLseFinThreads = 256;
constexpr int kLseFinCols = 32;
constexpr int kLseFinPhases = kLseFinThreads / kLseFinCols;

__global__ __launch_bounds__(kLseFinThreads) void lse_finalize_kernel(LseFinLaunch F) {
    __shared__ double sh[kLseFinPhases][kLseFinCols];
    __shared__ double red[2][kLseFinThreads / 64];
    const int tid = threadIdx.x;
    const int cl = tid % kLseFinCols;
    const int ph = tid / kLseFinCols;
    const int64_t j = (int64_t)blockIdx.x * kLseFinCols + cl;
    if (!F.marginal_only && ld_volatile_u32(&F.ctrl->done)) return;   // fixed for the whole launch
    const bool own = j < F.m;
    double M = -1e300;
    if (own)
        for (int w = ph; w < F.G; w += kLseFinPhases) M = fmax(M, F.pmax[(int64_t)w * F.ldp + j]);
    sh[ph][cl] = M;
    __syncthreads();
    M = sh[0][cl];
#pragma unroll
    for (int q = 1; q < kLseFinPhases; ++q) M = fmax(M, sh[q][cl]);
    __syncthreads();
    double S = 0.0;
    if (own)
        for (int w = ph; w < F.G; w += kLseFinPhases)
            S += (double)F.psum[(int64_t)w * F.ldp + j] *
                 (double)__builtin_amdgcn_exp2f((float)(F.pmax[(int64_t)w * F.ldp + j] - M));
    sh[ph][cl] = S;
    __syncthreads();
    double dn = 0.0, dc = 0.0;
    if (ph == 0 && own) {
        S = 0.0;
#pragma unroll
        for (int q = 0; q < kLseFinPhases; ++q) S += sh[q][cl];
        const double lse2 = S > 0.0 ? M + log2_pos(S) : -INFINITY;   // log2 sum_i 2^(F2_i - c C_ij)
        if (F.marginal_only) {
            const double G2 = F.c * F.g[j];
            F.c_out[j] = G2 == -INFINITY ? 0.0 : exp2_any(G2 + lse2);
        } else {
            const double lb = F.lb2[j];
            const double G2 = lb == -INFINITY ? -INFINITY : F.fi * (lb - lse2);
            F.g[j] = G2 * F.inv_c;
            const double cj = G2 == -INFINITY ? 0.0 : exp2_any(G2 + lse2);
            if (lb != -INFINITY && !(S > 0.0)) atomicOr(&F.ctrl->flags, UOT_FLAG_ZERO_SUM);
            if (lb != -INFINITY && !isfinite(G2)) atomicOr(&F.ctrl->flags, UOT_FLAG_NONFINITE);
            dn = fabs(cj - F.cprev[j]);
            dc = fabs(cj);
            F.cprev[j] = cj;
        }
    }
    if (F.marginal_only) return;
    dn = wave_sum_f64(dn);
    dc = wave_sum_f64(dc);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = dn;
        red[1][tid >> 6] = dc;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kLseFinThreads / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        F.blockpart[2 * blockIdx.x] = a;
        F.blockpart[2 * blockIdx.x + 1] = b;
    }
}

__global__ void lse_setup_kernel(const double* a, int64_t n, const double* b, int64_t m, double* la2, double* lb2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) la2[t] = a[t] > 0.0 ? log2(a[t]) : -INFINITY;
    else if (t - n < m) lb2[t - n] = b[t - n] > 0.0 ? log2(b[t - n]) : -INFINITY;
}

__global__ void cost_to_f32_kernel(const double* C, int64_t ldc, int64_t n, int64_t m, float* out, int64_t ldo) {
    const int64_t i = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ldo; j += (int64_t)gridDim.x * blockDim.x)
        out[i * ldo + j] = j < m ? (float)C[i * ldc + j] : 0.0f;
    (void)n;
}

int lse_finalize_blocks(int64_t m) { return (int)((m + kLseFinCols - 1) / kLseFinCols); }

int64_t lse_max_m(int c_dtype) {
    (void)c_dtype;
    return 8192;     // 8 FP64 or FP32 columns per lane: the exponents of a row stay in registers
}

hipError_t launch_lse_setup(const double* a, int64_t n, const double* b, int64_t m, double* la2, double* lb2,
                            hipStream_t stream) {
    const int64_t blocks = (n + m + 255) / 256;
    hipLaunchKernelGGL(lse_setup_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a, n, b, m, la2, lb2);
    return hipGetLastError();
}

hipError_t launch_cost_to_f32(const double* C, int64_t ldc, int64_t n, int64_t m, float* out, int64_t ldo,
                              hipStream_t stream) {
    const int64_t bx = std::min<int64_t>((ldo + 255) / 256, 64);
    hipLaunchKernelGGL(cost_to_f32_kernel, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, stream, C, ldc, n, m,
                       out, ldo);
    return hipGetLastError();
}

hipError_t launch_lse_finalize(const LseFinLaunch& F, hipStream_t stream) {
    hipLaunchKernelGGL(lse_finalize_kernel, dim3((unsigned)lse_finalize_blocks(F.m)), dim3(kLseFinThreads), 0,
                       stream, F);
    return hipGetLastError();
}

template <typename CT, int WG, int NC>
static hipError_t lse_launch_nc(int mode, const LseLaunch& L, hipStream_t stream) {
    constexpr int D = 2;
    const size_t lds = sizeof(double) * (size_t)WG * NC * (16 / sizeof(CT));
    auto kf = lse_kernel<CT, WG, NC, D, MODE_FUSED>;
    auto km = lse_kernel<CT, WG, NC, D, MODE_MARG>;
    auto kk = mode == MODE_FUSED ? kf : km;
    if (lds + 1024 > 65536) {     // with the static exchange arrays, beyond the default 64 KiB
        hipError_t e = hipFuncSetAttribute((const void*)kk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kk, dim3(L.P.grid), dim3(WG), lds, stream, L);
    return hipGetLastError();
}

// 512 lanes; chunks per lane: the fewest that cover the row (16 entries per
// lane at most: 8 FP64 chunks or 4 FP32 chunks, m <= 8192).
template <typename CT>
static hipError_t lse_launch_t(int mode, const LseLaunch& L, hipStream_t stream) {
    constexpr int64_t V = 16 / (int64_t)sizeof(CT);
    const int64_t per_chunk = kLseWG * V;
    if (L.P.m <= per_chunk) return lse_launch_nc<CT, kLseWG, 1>(mode, L, stream);
    if (L.P.m <= 2 * per_chunk) return lse_launch_nc<CT, kLseWG, 2>(mode, L, stream);
    if (L.P.m <= 4 * per_chunk) return lse_launch_nc<CT, kLseWG, 4>(mode, L, stream);
    if constexpr (V == 2)
        if (L.P.m <= 8 * per_chunk) return lse_launch_nc<CT, kLseWG, 8>(mode, L, stream);
    return hipErrorInvalidValue;
}

template <typename CT>
static int lse_occupancy_t(int64_t m) {
    constexpr int64_t V = 16 / (int64_t)sizeof(CT);
    const int64_t per_chunk = kLseWG * V;
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (m <= per_chunk)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lse_kernel<CT, kLseWG, 1, 2, MODE_FUSED>, kLseWG,
                                                         sizeof(double) * kLseWG * 1 * V);
    else if (m <= 2 * per_chunk)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lse_kernel<CT, kLseWG, 2, 2, MODE_FUSED>, kLseWG,
                                                         sizeof(double) * kLseWG * 2 * V);
    else if (m <= 4 * per_chunk)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lse_kernel<CT, kLseWG, 4, 2, MODE_FUSED>, kLseWG,
                                                         sizeof(double) * kLseWG * 4 * V);
    else if constexpr (V == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lse_kernel<CT, kLseWG, 8, 2, MODE_FUSED>, kLseWG,
                                                         sizeof(double) * kLseWG * 8 * V);
    return e == hipSuccess ? nb : 0;
}

int lse_wgs_per_cu(int c_dtype, int64_t m) {
    return c_dtype == UOT_F32 ? lse_occupancy_t<float>(m) : lse_occupancy_t<double>(m);
}

hipError_t launch_lse(int mode, const LseLaunch& L, hipStream_t stream) {
    if (mode != MODE_FUSED && mode != MODE_MARG) return hipErrorInvalidValue;
    if (L.c_dtype == UOT_F64) return lse_launch_t<double>(mode, L, stream);
    if (L.c_dtype == UOT_F32) return lse_launch_t<float>(mode, L, stream);
    return hipErrorInvalidValue;
}

}  // namespace uot
