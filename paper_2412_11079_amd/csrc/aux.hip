// O(n+m) steps of each iteration and the set-up / wrap-up kernels:
//   - column finalize (part 3 of the paper's split, Section 4, plus the
//     reduction of per-workgroup column partials that Algorithm 1 performs
//     after its thread join), with the stopping test of Section 2.1;
//   - initialisation, objective, cost from points, Gibbs kernel build.
#include "uot_common.h"

namespace uot {

// ---------------------------------------------------------------------------
// Initialisation
// ---------------------------------------------------------------------------
__global__ void init_kernel(double* u, int64_t n, const double* u0, double* v, int64_t m,
                            const double* v0, double* cprev, Ctrl* ctrl) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = t; i < n; i += stride) u[i] = u0 ? u0[i] : 1.0;
    for (int64_t j = t; j < m; j += stride) {
        v[j] = v0 ? v0[j] : 1.0;
        cprev[j] = 0.0;
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
// Block: 256 threads over 16 columns.  Thread t reads 4 adjacent columns
// (one 16-byte chunk) of strips t/4, t/4 + 64, ... with all loads of a
// group of 8 strips issued before any add; the 64 strip phases are then
// combined in LDS in a fixed order (one lane per column).
// ---------------------------------------------------------------------------
constexpr int FIN_COLS = 16;
constexpr int FIN_THREADS = 256;
constexpr int FIN_PHASES = FIN_THREADS / (FIN_COLS / 4);   // 64

int finalize_blocks(int64_t m) { return (int)((m + FIN_COLS - 1) / FIN_COLS); }

template <typename AT>
__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(FinLaunch F) {
    __shared__ double part[FIN_PHASES][FIN_COLS + 1];
    Ctrl* ctrl = F.ctrl;
    if (!F.marginal_only && ld_volatile_u32(&ctrl->done)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int cg = tid & (FIN_COLS / 4 - 1);   // 4-column group within the block
    const int ph = tid / (FIN_COLS / 4);       // strip phase
    const int64_t c0 = (int64_t)blockIdx.x * FIN_COLS + 4 * cg;
    const AT* P = (const AT*)F.partials + c0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (c0 < F.m) {
        // ldp is a multiple of 64, so the 4 columns never leave the partial row.
        constexpr int U = 8;
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

    // lanes >= FIN_COLS carry no column; they take part in the wave sums with zeros
    const int64_t j = (lane < FIN_COLS) ? (int64_t)blockIdx.x * FIN_COLS + lane : F.m;
    double w = 0.0;
    if (lane < FIN_COLS) {
#pragma unroll 16
        for (int k = 0; k < FIN_PHASES; ++k) w += part[k][lane];
    }

    double dsum = 0.0, csum = 0.0;
    if (j < F.m) {
        if (F.w_out) F.w_out[j] = w;
        if (F.marginal_only) {
            if (F.c_out) F.c_out[j] = F.v[j] * w;
            return;
        }
        const double bj = F.b[j];
        double shift = F.gpot ? -(1.0 - F.fi) * F.gpot[j] * F.inv_eps : 0.0;
        double vj = scale_factor(bj, w, F.fi, F.fi_is_one, shift);
        F.v[j] = vj;
        double cj = vj * w;
        double cp = F.cprev[j];
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
    for (int64_t i = tid; i < O.n; i += 1024) {
        double r = O.u[i] * O.s[i];
        if (O.r_out) O.r_out[i] = r;
        if (r > 0.0) sr += r * log(O.u[i]);
        mass += r;
        kr += kl_term(r, O.a[i]);
    }
    for (int64_t j = tid; j < O.m; j += 1024) {
        double c = O.v[j] * O.w[j];
        if (O.c_out) O.c_out[j] = c;
        if (c > 0.0) sc += c * log(O.v[j]);
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
            O.info->absorptions = 0;
            uint32_t fl = O.ctrl->flags;
            if (O.tol > 0.0 && !stopped && !(O.iters_run > 0 && stop_err <= O.tol)) fl |= UOT_FLAG_NOT_CONVERGED;
            if (!isfinite(L)) fl |= UOT_FLAG_NONFINITE;
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
template <typename KT>
__global__ void kernel_build(const double* __restrict__ C, int64_t ldc, int64_t n, int64_t m, double eps,
                             const double* __restrict__ f, const double* __restrict__ g,
                             KT* __restrict__ K, int64_t ldk) {
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double fi_ = f ? f[i] : 0.0;
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ldk;
             j += (int64_t)gridDim.x * blockDim.x) {
            KT val = (KT)0;
            if (j < m) {
                double e = fi_ - C[i * ldc + j];
                if (g) e += g[j];
                val = (KT)exp(e / eps);
            }
            K[i * ldk + j] = val;
        }
    }
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
                               hipStream_t stream) {
    dim3 grid = row_grid(n, ldk), block(256);
    if (k_dtype == UOT_F64)
        hipLaunchKernelGGL(kernel_build<double>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (double*)K, ldk);
    else if (k_dtype == UOT_F32)
        hipLaunchKernelGGL(kernel_build<float>, grid, block, 0, stream, C, ldc, n, m, eps, f, g, (float*)K, ldk);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace uot
