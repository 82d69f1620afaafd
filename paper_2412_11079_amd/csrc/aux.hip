// O(n+m) steps of each iteration and the set-up / wrap-up kernels:
//   - column finalize (part 3 of the paper's split, Section 4, plus the
//     reduction of per-workgroup column partials that Algorithm 1 performs
//     after its thread join), with the stopping test of Section 2.1;
//   - initialisation, objective, cost from points, Gibbs kernel build.
#include <algorithm>
#include <cmath>

#include "plan.h"
#include "uot_common.h"

namespace uot {

// ---------------------------------------------------------------------------
// Initialisation
// ---------------------------------------------------------------------------
__global__ void init_kernel(double* u, int64_t n, const double* u0, double* v, int64_t m,
                            const double* v0, double* cprev, Ctrl* ctrl) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (u)
        for (int64_t i = t; i < n; i += stride) u[i] = u0 ? u0[i] : 1.0;
    for (int64_t j = t; j < m; j += stride) {
        if (v) v[j] = v0 ? v0[j] : 1.0;
        if (cprev) cprev[j] = 0.0;
    }
    if (t == 0) {
        ctrl->done = 0;
        ctrl->bar = 0;
        ctrl->flags = 0;
        ctrl->pad0 = 0;
        ctrl->iters = 0;
        ctrl->err = 0.0;
    }
}

hipError_t launch_init(double* u, int64_t n, const double* u0, double* v, int64_t m, const double* v0,
                       double* cprev, Ctrl* ctrl, hipStream_t stream) {
    int64_t mx = n > m ? n : m;
    int blocks = (int)((mx + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, stream, u, n, u0, v, m, v0, cprev, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column finalize: w = sum over strips of the partials (fixed order, FP64),
// v = (b / w)^fi, c = v * w, and per-block sums of |c - c_prev| and |c| for
// the stopping test (evaluated by the next iteration's first pass).
// Block: 256 threads over 64 columns.  Thread t reads 4 adjacent columns
// (one 16-byte chunk) of strips t/16, t/16 + 16, ... with all loads of a
// group of 8 strips issued before any add; the 16 strip phases are then
// combined in LDS in a fixed order (one lane per column).
// ---------------------------------------------------------------------------
constexpr int FIN_COLS = 64;
constexpr int FIN_THREADS = 256;
constexpr int FIN_PHASES = FIN_THREADS / (FIN_COLS / 4);   // 16

int finalize_blocks(int64_t m) { return (int)((m + FIN_COLS - 1) / FIN_COLS); }

// Each wave reads 4 strips x 256 contiguous bytes per load; the per-column
// inputs and the stop flag are requested before the partials are summed so
// that their latency overlaps.
template <typename AT>
__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(FinLaunch F) {
    __shared__ double part[FIN_PHASES][FIN_COLS + 1];
    Ctrl* ctrl = F.ctrl;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int cg = tid & (FIN_COLS / 4 - 1);   // 4-column group within the block
    const int ph = tid / (FIN_COLS / 4);       // strip phase
    const int64_t c0 = (int64_t)blockIdx.x * FIN_COLS + 4 * cg;
    const int64_t j = (int64_t)blockIdx.x * FIN_COLS + lane;     // wave 0's column
    const bool own = wave == 0 && j < F.m;
    uint32_t done = 0;
    double bj = 0.0, cp = 0.0, gp = 0.0, vin = 0.0;
    if (own) {
        if (!F.marginal_only) {
            done = ld_volatile_u32(&ctrl->done);
            bj = F.b[j];
            cp = F.cprev[j];
            if (F.gpot) gp = F.gpot[j];
        } else if (F.c_out) {
            vin = F.v[j];
        }
    }
    const AT* P = (const AT*)F.partials + c0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (c0 < F.m) {
        // ldp is a multiple of 64, so the 4 columns never leave the partial row.
        constexpr int U = 16;
        int g = ph;
        for (; g + (U - 1) * FIN_PHASES < F.G; g += U * FIN_PHASES) {
            double x[U][4];
#pragma unroll
            for (int q = 0; q < U; ++q) Chunk4<AT>::load(P + (int64_t)(g + q * FIN_PHASES) * F.ldp, x[q]);
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[e] += x[q][e];
        }
        for (; g < F.G; g += FIN_PHASES) {
            double x[4];
            Chunk4<AT>::load(P + (int64_t)g * F.ldp, x);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += x[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[ph][4 * cg + e] = acc[e];
    __syncthreads();
    if (wave != 0) return;
    if (!F.marginal_only && __builtin_amdgcn_readfirstlane(done)) return;

    double w = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_PHASES; ++k) w += part[k][lane];
    w *= F.k_scale;

    double dsum = 0.0, csum = 0.0;
    if (own) {
        if (F.w_out) F.w_out[j] = w;
        if (F.marginal_only) {
            if (F.c_out) F.c_out[j] = vin * w;
            return;
        }
        double shift = F.gpot ? -(1.0 - F.fi) * gp * F.inv_eps : 0.0;
        double vj = scale_factor(bj, w, F.fi, F.fi_is_one, shift);
        F.v[j] = vj;
        double cj = vj * w;
        F.cprev[j] = cj;
        dsum = fabs(cj - cp);
        csum = fabs(cj);
        if (bj > 0.0 && !(w > 0.0)) atomicOr(&ctrl->flags, UOT_FLAG_ZERO_SUM);
        if (!isfinite(vj)) atomicOr(&ctrl->flags, UOT_FLAG_NONFINITE);
    }
    if (F.marginal_only) return;
    dsum = wave_sum_f64(dsum);
    csum = wave_sum_f64(csum);
    if (lane == 0) {
        F.blockpart[2 * blockIdx.x] = dsum;
        F.blockpart[2 * blockIdx.x + 1] = csum;
    }
}

hipError_t launch_finalize(const FinLaunch& F, hipStream_t stream) {
    dim3 grid(finalize_blocks(F.m)), block(FIN_THREADS);
    if (F.acc64)
        hipLaunchKernelGGL(finalize_kernel<double>, grid, block, 0, stream, F);
    else
        hipLaunchKernelGGL(finalize_kernel<float>, grid, block, 0, stream, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Objective (FP64, one workgroup, fixed reduction order):
//   L = eps (sum r log u + sum c log v - sum r) + tau KL~(r|a) + tau KL~(c|b)
// with r = u * (K v), c = v * (K^T u); valid because
// eps log P_ij = eps log u_i + eps log v_j - C_ij.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double kl_term(double x, double y) {
    double t = -x + y;
    if (x > 0.0) t += x * log(x / y);
    return t;
}

__global__ __launch_bounds__(1024) void objective_kernel(ObjLaunch O) {
    __shared__ double red[4][16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    double sr = 0.0, sc = 0.0, mass = 0.0, kr = 0.0, kc = 0.0;
    // With potentials, the total scalings are u e^{f/eps}, v e^{g/eps} and
    // log(total) = log u + f/eps; r = u * (Kt v), c = v * (Kt^T u) as before.
    const double inv_eps = 1.0 / O.eps;
    for (int64_t i = tid; i < (O.info_only ? 0 : O.n); i += 1024) {
        double r = O.u[i] * O.s[i];
        if (O.r_out) O.r_out[i] = r;
        double lu = (O.u[i] > 0.0) ? log(O.u[i]) + (O.fpot ? O.fpot[i] * inv_eps : 0.0) : -INFINITY;
        if (r > 0.0) sr += r * lu;
        if (O.f_out) O.f_out[i] = O.eps * lu;
        if (O.u_tot) O.u_tot[i] = (O.u[i] > 0.0) ? exp(lu) : 0.0;
        mass += r;
        kr += kl_term(r, O.a[i]);
    }
    for (int64_t j = tid; j < (O.info_only ? 0 : O.m); j += 1024) {
        double c = O.v[j] * O.w[j];
        if (O.c_out) O.c_out[j] = c;
        double lv = (O.v[j] > 0.0) ? log(O.v[j]) + (O.gpot ? O.gpot[j] * inv_eps : 0.0) : -INFINITY;
        if (c > 0.0) sc += c * lv;
        if (O.g_out) O.g_out[j] = O.eps * lv;
        if (O.v_tot) O.v_tot[j] = (O.v[j] > 0.0) ? exp(lv) : 0.0;
        kc += kl_term(c, O.b[j]);
    }
    double stop_err = 0.0;
    const bool stopped = O.ctrl->done != 0;
    if (wave == 0 && !stopped && O.iters_run > 0) stop_err = stop_error(O.blockpart, O.fin_blocks, lane);
    double vals[4] = {sr + sc - mass, kr, kc, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x = wave_sum_f64(vals[q]);
        if (lane == 0) red[q][wave] = x;
    }
    __syncthreads();
    if (tid == 0) {
        double e = 0.0, a = 0.0, b = 0.0;
        for (int w = 0; w < 16; ++w) {
            e += red[0][w];
            a += red[1][w];
            b += red[2][w];
        }
        double L = O.eps * e;
        if (!O.tau_inf) L += O.tau * (a + b);
        if (O.loss) *O.loss = L;
        if (O.info) {
            // Stopped: the pass that found err <= tol recorded it.  Otherwise
            // all enqueued iterations ran; the last one may still meet tol.
            O.info->iters = stopped ? O.ctrl->iters : O.iters_run;
            O.info->err = stopped ? O.ctrl->err : stop_err;
            O.info->absorptions = O.absorptions;
            uint32_t fl = O.ctrl->flags;
            if (O.tol > 0.0 && !stopped && !(O.iters_run > 0 && stop_err <= O.tol)) fl |= UOT_FLAG_NOT_CONVERGED;
            if (!O.info_only && !isfinite(L)) fl |= UOT_FLAG_NONFINITE;
            O.info->flags = fl;
        }
    }
}

hipError_t launch_objective(const ObjLaunch& O, hipStream_t stream) {
    hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(1024), 0, stream, O);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cost from points: 32 x 32 output tiles, points staged through LDS in
// slices of 16 coordinates; FP64 throughout.  Per-block maxima go to
// blockmax; normalisation divides by the maximum of those.
// ---------------------------------------------------------------------------
constexpr int CT = 32;     // tile edge
constexpr int CD = 16;     // coordinates per LDS slice

int64_t cost_blocks(int64_t n, int64_t m) { return ((n + CT - 1) / CT) * ((m + CT - 1) / CT); }

__global__ __launch_bounds__(256) void cost_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                   int64_t n, int64_t m, int64_t d, int kind,
                                                   double* __restrict__ C, int64_t ldc,
                                                   double* __restrict__ blockmax) {
    __shared__ double xs[CT][CD + 1];
    __shared__ double ys[CT][CD + 1];
    __shared__ double wmax[4];
    const int tx = threadIdx.x & 31;      // column within tile
    const int ty = threadIdx.x >> 5;      // 0..7: rows ty, ty+8, ty+16, ty+24
    const int64_t tiles_m = (m + CT - 1) / CT;
    const int64_t bi = blockIdx.x / tiles_m, bj = blockIdx.x % tiles_m;
    const int64_t i0 = bi * CT, j0 = bj * CT;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < d; k0 += CD) {
        for (int t = threadIdx.x; t < CT * CD; t += 256) {
            int rr = t / CD, kk = t % CD;
            int64_t gi = i0 + rr, gj = j0 + rr, gk = k0 + kk;
            xs[rr][kk] = (gi < n && gk < d) ? x[gi * d + gk] : 0.0;
            ys[rr][kk] = (gj < m && gk < d) ? y[gj * d + gk] : 0.0;
        }
        __syncthreads();
        int kmax = (int)((d - k0) < CD ? (d - k0) : CD);
        for (int kk = 0; kk < kmax; ++kk) {
            double yv = ys[tx][kk];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double xv = xs[ty + 8 * q][kk];
                if (kind == UOT_COST_SQEUCLID) {
                    double diff = xv - yv;
                    acc[q] += diff * diff;
                } else {
                    acc[q] += xv * yv;
                }
            }
        }
        __syncthreads();
    }
    double mx = -INFINITY;
    const int64_t gj = j0 + tx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t gi = i0 + ty + 8 * q;
        if (gi < n && gj < m) {
            double val = (kind == UOT_COST_SQEUCLID) ? acc[q] : 1.0 - acc[q];
            C[gi * ldc + gj] = val;
            mx = fmax(mx, val);
        }
    }
    mx = wave_max_f64(mx);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0 && blockmax)
        blockmax[blockIdx.x] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}

__global__ __launch_bounds__(1024) void max_reduce_kernel(double* blockmax, int64_t count) {
    __shared__ double wm[16];
    double mx = -INFINITY;
    for (int64_t k = threadIdx.x; k < count; k += 1024) mx = fmax(mx, blockmax[k]);
    mx = wave_max_f64(mx);
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = wm[0];
        for (int w = 1; w < 16; ++w) r = fmax(r, wm[w]);
        blockmax[count] = r;     // the global maximum lands after the block maxima
    }
}

__global__ void scale_kernel(double* C, int64_t n, int64_t m, int64_t ldc, const double* gmax) {
    const double mx = *gmax;
    if (!(mx > 0.0)) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
             j += (int64_t)gridDim.x * blockDim.x)
            C[i * ldc + j] = C[i * ldc + j] / mx;
}

hipError_t launch_cost(const double* x, const double* y, int64_t n, int64_t m, int64_t d, int kind,
                       int normalize, double* C, int64_t ldc, double* blockmax, hipStream_t stream) {
    int64_t nb = cost_blocks(n, m);
    hipLaunchKernelGGL(cost_kernel, dim3((unsigned)nb), dim3(256), 0, stream, x, y, n, m, d, kind, C, ldc,
                       blockmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !normalize) return e;
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(1024), 0, stream, blockmax, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t gx = (m + 255) / 256 < 64 ? (m + 255) / 256 : 64;
    int64_t gy = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, stream, C, n, m, ldc,
                       blockmax + nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gibbs kernel K_ij = RNE(exp((f_i + g_j - C_ij)/eps)) from FP64, padding
// columns [m, ldk) written as 0.
// ---------------------------------------------------------------------------
// grid.y strides over rows, grid.x * 256 threads over the columns of a row.
template <typename KT> struct Store;
template <> struct Store<double> {
    static __device__ __forceinline__ double cv(double x) { return x; }
};
template <> struct Store<float> {
    static __device__ __forceinline__ float cv(double x) { return (float)x; }
};
template <> struct Store<bf16_t> {
    static __device__ __forceinline__ bf16_t cv(double x) { return bf16_t{f64_to_bf16(x)}; }
};
template <> struct Store<fp8_t> {
    static __device__ __forceinline__ fp8_t cv(double x) { return fp8_t{f64_to_e4m3(x)}; }
};

// Four adjacent stored entries written with one store (4-entry chunks start
// at a multiple of 4 entries and rows at a multiple of 16 bytes).
template <typename KT> struct Pack4;
template <> struct Pack4<double> {
    static __device__ __forceinline__ void put(double* p, const double* x) {
        *(f64x2*)p = f64x2{x[0], x[1]};
        *(f64x2*)(p + 2) = f64x2{x[2], x[3]};
    }
};
template <> struct Pack4<float> {
    static __device__ __forceinline__ void put(float* p, const double* x) {
        *(f32x4*)p = f32x4{(float)x[0], (float)x[1], (float)x[2], (float)x[3]};
    }
};
template <> struct Pack4<bf16_t> {
    static __device__ __forceinline__ void put(bf16_t* p, const double* x) {
        uint64_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (uint64_t)f64_to_bf16(x[e]) << (16 * e);
        *(uint64_t*)p = w;
    }
};
template <> struct Pack4<fp8_t> {
    static __device__ __forceinline__ void put(fp8_t* p, const double* x) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (uint32_t)f64_to_e4m3(x[e]) << (8 * e);
        *(uint32_t*)p = w;
    }
};

// Each lane builds 4 adjacent entries of a row.  Exponents e = f_i + g_j -
// C_ij below `cut` are stored as 0 without evaluating exp: cut sits a factor
// e below the largest value the storage type rounds to zero (see zero_cut),
// so the stored bits are the same.
template <typename KT>
__global__ void kernel_build(const double* __restrict__ C, int64_t ldc, int64_t n, int64_t m, double eps,
                             const double* __restrict__ f, const double* __restrict__ g,
                             KT* __restrict__ K, int64_t ldk, double store_scale, double cut) {
    const int64_t chunks = (ldk + 3) / 4;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double fi_ = f ? f[i] : 0.0;
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < chunks;
             q += (int64_t)gridDim.x * blockDim.x) {
            const int64_t j0 = 4 * q;
            // C's four entries as two 16-byte loads where the row allows it
            const double* crow = C + i * ldc + j0;
            double cv[4];
            if (j0 + 4 <= m && ((uintptr_t)crow & 15) == 0) {
                const f64x2 c01 = *(const f64x2*)crow;
                const f64x2 c23 = *(const f64x2*)(crow + 2);
                cv[0] = c01[0];
                cv[1] = c01[1];
                cv[2] = c23[0];
                cv[3] = c23[1];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) cv[e] = j0 + e < m ? crow[e] : 0.0;
            }
            double val[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = j0 + e;
                val[e] = 0.0;
                if (j < m) {
                    double x = fi_ - cv[e];
                    if (g) x += g[j];
                    if (!(x < cut)) val[e] = store_scale * exp(x / eps);
                }
            }
            KT* p = K + i * ldk + j0;
            if (j0 + 4 <= ldk) {
                Pack4<KT>::put(p, val);
            } else {
                for (int e = 0; j0 + e < ldk; ++e) p[e] = Store<KT>::cv(val[e]);
            }
        }
    }
}

// Exponent below which store_scale * exp(e / eps) certainly stores as 0:
// the type's zero bound (FP64: exp underflows below 2^-1075; FP32: values up
// to 2^-150 round to 0; BF16 here: below 2^-126; E4M3: up to 2^-10), one
// unit of e / eps further down so that rounding of exp and of this bound
// cannot matter.
static double zero_cut(int k_dtype, double eps, double store_scale) {
    if (!(store_scale > 0.0) || !(eps > 0.0)) return -INFINITY;
    double lb;
    switch (k_dtype) {
        case UOT_F64: lb = -1075.0; break;
        case UOT_F32: lb = -150.0; break;
        case UOT_BF16: lb = -126.0; break;
        case UOT_FP8_E4M3: lb = -10.0; break;
        default: return -INFINITY;
    }
    return (lb * std::log(2.0) - std::log(store_scale) - 1.0) * eps;
}

static dim3 row_grid(int64_t n, int64_t cols) {
    int64_t gx = (cols + 255) / 256;
    if (gx > 64) gx = 64;
    int64_t gy = n < 4096 ? n : 4096;
    if (gx < 1) gx = 1;
    if (gy < 1) gy = 1;
    return dim3((unsigned)gx, (unsigned)gy);
}

hipError_t launch_kernel_build(const double* C, int64_t ldc, int64_t n, int64_t m, double eps,
                               const double* f, const double* g, int k_dtype, void* K, int64_t ldk,
                               double store_scale, hipStream_t stream) {
    dim3 grid = row_grid(n, (ldk + 3) / 4), block(256);
    const double cut = zero_cut(k_dtype, eps, store_scale);
    switch (k_dtype) {
        case UOT_F64:
            hipLaunchKernelGGL(kernel_build<double>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (double*)K, ldk,
                               store_scale, cut);
            break;
        case UOT_F32:
            hipLaunchKernelGGL(kernel_build<float>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (float*)K, ldk,
                               store_scale, cut);
            break;
        case UOT_BF16:
            hipLaunchKernelGGL(kernel_build<bf16_t>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (bf16_t*)K,
                               ldk, store_scale, cut);
            break;
        case UOT_FP8_E4M3:
            hipLaunchKernelGGL(kernel_build<fp8_t>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (fp8_t*)K, ldk,
                               store_scale, cut);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stabilised (absorbed) kernel rebuild.  With
//   f_i = min_j (C_ij - g_j)      then      g_j <- min_i (C_ij - f_i)  (>= g_j)
// every exponent f_i + g_j - C_ij is <= 0, every column reaches 0 and every
// row still does (at its own minimum), so Kt = exp((f + g - C)/eps) has
// row and column maxima exactly 1: each stored type keeps each row's and
// column's largest entries at full precision and no column is flushed
// whole.  u and v are rescaled so the totals u e^{f/eps}, v e^{g/eps} are
// unchanged (on the first build u and v hold the totals: f_old = g_old = 0).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void rowmin_kernel(const double* __restrict__ C, int64_t ldc, int64_t n,
                                                     int64_t m, double eps, double* __restrict__ f,
                                                     const double* __restrict__ g, double* __restrict__ u,
                                                     int first) {
    __shared__ double wmin[4];
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const double* Ci = C + i * ldc;
        double mn = INFINITY;
        for (int64_t j = threadIdx.x; j < m; j += 256) mn = fmin(mn, Ci[j] - g[j]);
        // min is order independent: any reduction order gives the same bits
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, 64));
        if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = mn;
        __syncthreads();
        const double fnew = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
        __syncthreads();
        if (threadIdx.x == 0) {
            const double fold = first ? 0.0 : f[i];
            if (u[i] > 0.0) u[i] = exp(log(u[i]) + (fold - fnew) / eps);
            f[i] = fnew;
        }
    }
}

// Order-preserving map of a double to an unsigned key (negative values:
// all bits flipped; others: the sign bit set), so that an integer atomic
// min over keys is the exact FP64 minimum, independent of arrival order.
__device__ __forceinline__ unsigned long long min_key(double d) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double min_key_value(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Column minima of C_ij - f_i (of either sign: g takes absorbed values).
__global__ __launch_bounds__(256) void colmin_kernel(const double* __restrict__ C, int64_t ldc, int64_t n,
                                                     int64_t m, const double* __restrict__ f,
                                                     unsigned long long* __restrict__ gmin_keys, int64_t rows_per_block) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int64_t i0 = (int64_t)blockIdx.y * rows_per_block;
    int64_t i1 = i0 + rows_per_block;
    if (i1 > n) i1 = n;
    double mn = INFINITY;
    for (int64_t i = i0; i < i1; ++i) mn = fmin(mn, C[i * ldc + j] - f[i]);
    atomicMin(&gmin_keys[j], min_key(mn));
}

// Row and column minima in one read of C, for rows of up to 1024 CPT
// columns.  Each 1024-lane workgroup takes a strip of rows; a row is held in
// registers (lane t: columns t, t + 1024, ...) while the next row's loads
// are in flight; g sits in LDS.  Its minimum of C_ij - g_j gives f_i (u_i is rescaled as in
// rowmin_kernel), and the same registers then update the lane's running
// minima of C_ij - f_i, which go to the column keys with one atomic min per
// column at the end.  The results equal those of the two separate kernels:
// a minimum does not depend on the order it is taken in.
template <int CPT>
__global__ __launch_bounds__(1024) void rowcolmin_kernel(const double* __restrict__ C, int64_t ldc, int64_t n,
                                                         int64_t m, double eps, double* __restrict__ f,
                                                         const double* __restrict__ g, double* __restrict__ u,
                                                         int first, unsigned long long* __restrict__ gmin_keys,
                                                         int64_t rows_per_block) {
    __shared__ double wmin[2][16];
    extern __shared__ double gsh[];            // g, 1024 CPT entries
    const int t = threadIdx.x;
    double cmin[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t j = (int64_t)c * 1024 + t;
        gsh[c * 1024 + t] = j < m ? g[j] : 0.0;
        cmin[c] = INFINITY;
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t i1 = i0 + rows_per_block;
    if (i1 > n) i1 = n;
    double x[2][CPT];
    auto load = [&](int q, int64_t i) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int64_t j = (int64_t)c * 1024 + t;
            x[q][c] = (j < m && i < i1) ? C[i * ldc + j] : INFINITY;
        }
    };
    int slot = 0;
    auto row = [&](int q, int64_t i) {
        double mn = INFINITY;
#pragma unroll
        for (int c = 0; c < CPT; ++c) mn = fmin(mn, x[q][c] - gsh[c * 1024 + t]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, 64));
        if ((t & 63) == 0) wmin[slot][t >> 6] = mn;
        __syncthreads();
        double fnew = wmin[slot][0];
#pragma unroll
        for (int w = 1; w < 16; ++w) fnew = fmin(fnew, wmin[slot][w]);
        slot ^= 1;
        if (t == 0) {
            const double fold = first ? 0.0 : f[i];
            if (u[i] > 0.0) u[i] = exp(log(u[i]) + (fold - fnew) / eps);
            f[i] = fnew;
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) cmin[c] = fmin(cmin[c], x[q][c] - fnew);
    };
    load(0, i0);
    for (int64_t i = i0; i < i1; i += 2) {
        load(1, i + 1);
        row(0, i);
        if (i + 1 >= i1) break;
        load(0, i + 2);
        row(1, i + 1);
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t j = (int64_t)c * 1024 + t;
        if (j < m && i1 > i0) atomicMin(&gmin_keys[j], min_key(cmin[c]));
    }
}

__global__ void fill_bits_kernel(unsigned long long* p, int64_t count, unsigned long long bits) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = bits;
}

// g_j <- the column minimum, v_j rescaled to keep v e^{g/eps}.
__global__ void gshift_kernel(const unsigned long long* __restrict__ gmin_keys, double* __restrict__ g,
                              double* __restrict__ v, int64_t m, double eps, int first) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const double gnew = min_key_value(gmin_keys[j]);
        const double gold = first ? 0.0 : g[j];
        if (v[j] > 0.0) v[j] = exp(log(v[j]) + (gold - gnew) / eps);
        g[j] = gnew;
    }
}

hipError_t launch_rebuild(const double* C, int64_t ldc, int64_t n, int64_t m, double eps, double* f, double* g,
                          double* u, double* v, void* gmin_scratch, int k_dtype, void* K, int64_t ldk,
                          double store_scale, int first, hipStream_t stream) {
    unsigned long long* gb = (unsigned long long*)gmin_scratch;
    const unsigned long long inf_bits = 0xfff0000000000000ull;   // min_key(+inf)
    int fb = (int)((m + 255) / 256);
    if (fb > 1024) fb = 1024;
    hipLaunchKernelGGL(fill_bits_kernel, dim3(fb), dim3(256), 0, stream, gb, m, inf_bits);
    if (m <= 1024 * 8) {
        // one read of C, one strip per CU
        const int64_t rpb = (n + 255) / 256;
        const unsigned blocks = (unsigned)((n + rpb - 1) / rpb);
        if (m <= 1024 * 2)
            hipLaunchKernelGGL(rowcolmin_kernel<2>, dim3(blocks), dim3(1024), 2 * 1024 * sizeof(double), stream, C,
                               ldc, n, m, eps, f, g, u, first, gb, rpb);
        else if (m <= 1024 * 4)
            hipLaunchKernelGGL(rowcolmin_kernel<4>, dim3(blocks), dim3(1024), 4 * 1024 * sizeof(double), stream, C,
                               ldc, n, m, eps, f, g, u, first, gb, rpb);
        else
            hipLaunchKernelGGL(rowcolmin_kernel<8>, dim3(blocks), dim3(1024), 8 * 1024 * sizeof(double), stream, C,
                               ldc, n, m, eps, f, g, u, first, gb, rpb);
    } else {
        const int rblocks = (int)(n < 65536 ? n : 65536);
        hipLaunchKernelGGL(rowmin_kernel, dim3(rblocks), dim3(256), 0, stream, C, ldc, n, m, eps, f, g, u, first);
        const int64_t rows_per_block = 256;
        dim3 cgrid((unsigned)((m + 255) / 256), (unsigned)((n + rows_per_block - 1) / rows_per_block));
        hipLaunchKernelGGL(colmin_kernel, cgrid, dim3(256), 0, stream, C, ldc, n, m, f, gb, rows_per_block);
    }
    hipLaunchKernelGGL(gshift_kernel, dim3(fb), dim3(256), 0, stream, gb, g, v, m, eps, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_kernel_build(C, ldc, n, m, eps, f, g, k_dtype, K, ldk, store_scale, stream);
}

// max |log u_i| and max |log v_j| (over positive entries) into out[0], out[1]
// as the bit patterns of non-negative doubles, whose unsigned order is their
// numeric order: each workgroup takes a slice and atomically maxes its result
// (exact and order independent).  out must start at +0.
__global__ __launch_bounds__(256) void absorb_check_kernel(const double* u, int64_t n, const double* v, int64_t m,
                                                          unsigned long long* out) {
    __shared__ double red[2][4];
    double mu = 0.0, mv = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        if (u[i] > 0.0) mu = fmax(mu, fabs(log(u[i])));
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += stride)
        if (v[j] > 0.0) mv = fmax(mv, fabs(log(v[j])));
    mu = wave_max_f64(mu);
    mv = wave_max_f64(mv);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = mu;
        red[1][threadIdx.x >> 6] = mv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < 4; ++w) {
            a = fmax(a, red[0][w]);
            b = fmax(b, red[1][w]);
        }
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(a));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(b));
    }
}

hipError_t launch_absorb_check(const double* u, int64_t n, const double* v, int64_t m, double* out,
                               hipStream_t stream) {
    unsigned long long* keys = (unsigned long long*)out;
    hipLaunchKernelGGL(fill_bits_kernel, dim3(1), dim3(64), 0, stream, keys, (int64_t)2, 0ull);
    int64_t blocks = (std::max(n, m) + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(absorb_check_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, u, n, v, m, keys);
    return hipGetLastError();
}

__global__ void absorb_apply_kernel(double* v, double* g, int64_t m, double eps) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        if (v[j] > 0.0) {
            g[j] += eps * log(v[j]);
            v[j] = 1.0;
        }
    }
}

hipError_t launch_absorb_apply(double* v, double* g, int64_t m, double eps, hipStream_t stream) {
    int blocks = (int)((m + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(absorb_apply_kernel, dim3(blocks), dim3(256), 0, stream, v, g, m, eps);
    return hipGetLastError();
}

// Decode stored K (16-byte chunks, count a multiple of the chunk size) to FP32.
template <typename KT>
__global__ void decode_kernel(const KT* K, int64_t chunks, double scale, float* out) {
    using Raw = typename KVec<KT>::raw;
    constexpr int V = KVec<KT>::N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < chunks; t += (int64_t)gridDim.x * blockDim.x) {
        Raw r = ((const Raw*)K)[t];
        float x[V];
        Unpack<KT, float>::run(r, x);
#pragma unroll
        for (int e = 0; e < V; ++e) out[t * V + e] = (float)(scale * x[e]);
    }
}

hipError_t launch_decode(const void* K, int k_dtype, int64_t count, double scale, float* out, hipStream_t stream) {
    dim3 grid(1024), block(256);
    switch (k_dtype) {
        case UOT_F64: hipLaunchKernelGGL(decode_kernel<double>, grid, block, 0, stream, (const double*)K, count / 2, scale, out); break;
        case UOT_F32: hipLaunchKernelGGL(decode_kernel<float>, grid, block, 0, stream, (const float*)K, count / 4, scale, out); break;
        case UOT_BF16: hipLaunchKernelGGL(decode_kernel<bf16_t>, grid, block, 0, stream, (const bf16_t*)K, count / 8, scale, out); break;
        case UOT_FP8_E4M3: hipLaunchKernelGGL(decode_kernel<fp8_t>, grid, block, 0, stream, (const fp8_t*)K, count / 16, scale, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense plan P = diag(u) K diag(v) (from a stored K and the scalings), or
// P = exp((f_i + g_j - C_ij)/eps) (from the cost and the potentials of the
// total scalings, the form that stays finite when u, v overflow).  One
// 2-D grid: y over rows, x over 16-byte chunks of K / columns.
// ---------------------------------------------------------------------------
template <typename KT, typename PT>
__global__ __launch_bounds__(256) void plan_from_k_kernel(const KT* __restrict__ K, int64_t ldk, int64_t n,
                                                          int64_t m, double k_scale, const double* __restrict__ u,
                                                          const double* __restrict__ v, PT* __restrict__ P,
                                                          int64_t ldp, const double* __restrict__ dscale) {
    using Raw = typename KVec<KT>::raw;
    constexpr int V = KVec<KT>::N;
    const int64_t chunks = (m + V - 1) / V;
    const double sc = dscale ? k_scale * *dscale : k_scale;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double ui = u[i] * sc;
        const Raw* row = (const Raw*)(K + i * ldk);
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256) {
            double x[V];
            Unpack<KT, double>::run(row[q], x);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t j = q * V + e;
                if (j < m) P[i * ldp + j] = (PT)(ui * x[e] * v[j]);
            }
        }
    }
}

template <typename PT>
__global__ __launch_bounds__(256) void plan_from_cost_kernel(const double* __restrict__ C, int64_t ldc, int64_t n,
                                                             int64_t m, double eps, const double* __restrict__ f,
                                                             const double* __restrict__ g, PT* __restrict__ P,
                                                             int64_t ldp) {
    const double inv_eps = 1.0 / eps;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double fi = f[i];
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)gridDim.x * 256)
            P[i * ldp + j] = (PT)exp((fi + g[j] - C[i * ldc + j]) * inv_eps);
    }
}

template <typename PT>
static hipError_t launch_plan_k_typed(const void* K, int k_dtype, int64_t ldk, int64_t n, int64_t m, double k_scale,
                                      const double* u, const double* v, PT* P, int64_t ldp, const double* dscale,
                                      hipStream_t stream) {
    const int64_t chunks_max = (m + 1) / 2;
    dim3 grid((unsigned)std::min<int64_t>((chunks_max + 255) / 256, 64), (unsigned)std::min<int64_t>(n, 4096));
    switch (k_dtype) {
        case UOT_F64: hipLaunchKernelGGL((plan_from_k_kernel<double, PT>), grid, dim3(256), 0, stream, (const double*)K, ldk, n, m, k_scale, u, v, P, ldp, dscale); break;
        case UOT_F32: hipLaunchKernelGGL((plan_from_k_kernel<float, PT>), grid, dim3(256), 0, stream, (const float*)K, ldk, n, m, k_scale, u, v, P, ldp, dscale); break;
        case UOT_BF16: hipLaunchKernelGGL((plan_from_k_kernel<bf16_t, PT>), grid, dim3(256), 0, stream, (const bf16_t*)K, ldk, n, m, k_scale, u, v, P, ldp, dscale); break;
        case UOT_FP8_E4M3: hipLaunchKernelGGL((plan_from_k_kernel<fp8_t, PT>), grid, dim3(256), 0, stream, (const fp8_t*)K, ldk, n, m, k_scale, u, v, P, ldp, dscale); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_plan_from_k(const void* K, int k_dtype, int64_t ldk, int64_t n, int64_t m, double k_scale,
                              const double* u, const double* v, void* P, int plan_dtype, int64_t ldp,
                              hipStream_t stream, const double* dscale) {
    if (plan_dtype == UOT_F64)
        return launch_plan_k_typed<double>(K, k_dtype, ldk, n, m, k_scale, u, v, (double*)P, ldp, dscale, stream);
    if (plan_dtype == UOT_F32)
        return launch_plan_k_typed<float>(K, k_dtype, ldk, n, m, k_scale, u, v, (float*)P, ldp, dscale, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_plan_from_cost(const double* C, int64_t ldc, int64_t n, int64_t m, double eps, const double* f,
                                 const double* g, void* P, int plan_dtype, int64_t ldp, hipStream_t stream) {
    dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)std::min<int64_t>(n, 4096));
    if (plan_dtype == UOT_F64)
        hipLaunchKernelGGL(plan_from_cost_kernel<double>, grid, dim3(256), 0, stream, C, ldc, n, m, eps, f, g, (double*)P, ldp);
    else if (plan_dtype == UOT_F32)
        hipLaunchKernelGGL(plan_from_cost_kernel<float>, grid, dim3(256), 0, stream, C, ldc, n, m, eps, f, g, (float*)P, ldp);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace uot
