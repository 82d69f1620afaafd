// Batched UOT Sinkhorn: many independent problems of uneven size in one
// persistent launch.
//
// Every workgroup (256 lanes, four waves) takes problems from a queue in
// longest-first order and runs all iterations of a problem by itself: the
// row half-step and the column accumulation happen in one pass over the
// problem's K per iteration (the single-pass interleave of the paper's
// Section 4.1, here inside one workgroup), the column sums never leave the
// workgroup, and v lives in LDS between iterations.  No grid-wide
// synchronisation exists, so the launch is a plain kernel that a HIP graph
// can hold.
//
// Tile shape of a problem (BatchDesc::shape, chosen per problem on the
// host): rg row groups of 256/rg lanes work on rg rows at once (rg = 4: one
// wave per row and no barrier per row), and each lane covers nc 16-byte
// chunks of a row (at most kLaneCols values).  The shape is a run-time
// value, so one code path serves every problem.  Arithmetic: products, row
// sums and column sums in FP64 (the stored K is widened), so a problem's
// result is the FP64 iteration on its stored K up to summation order.
#include <math.h>

#include "batch.h"
#include "scalemath.h"
#include "strip.h"

namespace uot {

namespace {

constexpr int kBatchWG = 256;
constexpr int kBatchNW = kBatchWG / 64;

struct BatchShapeDef {
    int rg;
    int nc;
};
constexpr BatchShapeDef kBatchShapes[] = {{4, 1}, {4, 2}, {4, 4}, {2, 1}, {2, 2}, {2, 4}, {1, 1}, {1, 2}, {1, 4}};
constexpr int kNumBatchShapes = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);
constexpr int kLaneCols = 8;            // FP64 column sums a lane holds

template <typename KT>
constexpr int nc_max() {
    return KVec<KT>::N >= kLaneCols ? 1 : kLaneCols / KVec<KT>::N;
}

// Rows per batch of a row group: the batch's dots are reduced together,
// with one LDS exchange, and its R scaling factors are computed side by
// side (lane r of each wave evaluates row r), so the long FP64 chain of the
// power is paid once per batch, not once per row.  Two batches are in
// registers (one being processed, the next one loading).  A problem's time
// follows its batch count, so R is as large as the registers allow (FP32:
// 6, measured against 3, 4 and 5; a few spilled values cost less than the
// batches saved).
constexpr int kBatchMaxRows = 8;
template <typename KT>
constexpr int rows_per_batch() {
    if (nc_max<KT>() >= 4 || KVec<KT>::N >= 16) return 2;      // FP64, FP8: within 256 VGPRs
    return KVec<KT>::N == 4 ? 6 : 4;                            // FP32, BF16
}

// Block-wide FP64 sum in a fixed order; every thread receives the result.
__device__ __forceinline__ double block_sum(double x, double* scratch) {
    x = wave_sum_f64(x);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[wave] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBatchNW; ++w) t += scratch[w];
    return t;
}

// Barrier of the parts of a split problem (workgroups on any XCD): each
// part adds 1 to the problem's counter once its column sums are written,
// then waits until all P parts of this round have arrived (target P t in
// round t).  Release and acquire at agent scope around the counter make the
// sums visible across L2s; the wait is bounded (flag on timeout).
__device__ __forceinline__ void part_barrier(uint32_t* hdr, uint32_t target) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&hdr[0], 1u);
        uint32_t spins = 0;
        while (__hip_atomic_load(&hdr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kBarrierSpinLimit) {
                atomicOr(&hdr[1], UOT_FLAG_BARRIER_TIMEOUT);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// (target / sum)^fi in FP64 with the log and exp of scalemath.h, whose
// coefficients stay in scalar registers: the library routines would hold
// theirs in vector registers across the whole problem loop.  Special
// quotients follow the plain formula (0 -> 0, +inf -> +inf, NaN -> NaN).
__device__ __forceinline__ double batch_factor(double target, double sum, double fi, int fi_is_one) {
    if (target == 0.0) return 0.0;
    const double q = target / sum;
    if (fi_is_one || !(q > 0.0) || q == INFINITY) return q;
    return sm::exp_any(fi * sm::log_pos(q));
}

__device__ __forceinline__ double kl_term(double x, double y) {
    // x log(x/y) - x + y with 0 log 0 = 0
    if (x > 0.0) return x * log(x / y) - x + y;
    return y;
}

struct BatchShared {
    double red[2][kBatchMaxRows][kBatchNW];
    double scratch[kBatchNW];
    int32_t idx;
    uint32_t flags;
};

template <typename KT>
struct BatchSolve {
    using KV = KVec<KT>;
    using Raw = typename KV::raw;
    static constexpr int V = KV::N;
    static constexpr int NCM = nc_max<KT>();
    static constexpr int E = NCM * V;
    static constexpr int R = rows_per_batch<KT>();
    static_assert(R <= kBatchMaxRows, "row exchange holds kBatchMaxRows rows");

    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t row_bytes;
    int rg, nc, lr, wpr, grp, gl;
    int col[NCM];                       // first column of each chunk (m < 2^31)
    uint32_t voff[NCM];
    Raw buf[2][R][NCM];
    double abuf[2];                     // a of the batch row lane r (r < R) holds, loaded with the rows
    const double* pa;
    int64_t pn;
    double acc[E];

    // Rows k = b R + r (r < R) of the group, i = grp + rg k, into buffer Q;
    // rows beyond the matrix read 0.
    template <int Q>
    __device__ __forceinline__ void load_batch(int64_t b) {
        const int lane = threadIdx.x & 63;
        const int64_t il = grp + (int64_t)rg * (b * R + (lane < R ? lane : 0));
        abuf[Q] = (lane < R && il < pn) ? pa[il] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t soff = (uint32_t)(grp + (int64_t)rg * (b * R + r)) * row_bytes;
#pragma unroll
            for (int c = 0; c < NCM; ++c)
                buf[Q][r][c] = __builtin_bit_cast(
                    Raw, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(voff[c] + soff), 0, 2));
        }
    }

    // The lane's chunk c of row r in buffer Q, widened; columns >= m read
    // as 0 (chunks beyond the shape's nc point past the buffer and read 0).
    template <int Q>
    __device__ __forceinline__ void unpack(int r, int c, int m, bool ragged, double* x) const {
        Unpack<KT, double>::run(buf[Q][r][c], x);
        if (ragged) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (col[c] + e >= m) x[e] = 0.0;
        }
    }

    // The same chunk widened afresh for the column update: the opaque copy
    // keeps the compiler from holding the row dot's widened values (twice
    // the registers of the stored ones) across the scaling factors.
    template <int Q>
    __device__ __forceinline__ void unpack_again(int r, int c, int m, bool ragged, double* x) const {
        Raw q = buf[Q][r][c];
        asm volatile("" : "+v"(q));
        Unpack<KT, double>::run(q, x);
        if (ragged) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (col[c] + e >= m) x[e] = 0.0;
        }
    }

    // Row totals of the batch (every lane of the group gets all R).
    template <int Q>
    __device__ __forceinline__ void batch_totals(const double* vl, int m, bool ragged, BatchShared& sh, int& slot,
                                                 double* t) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < NCM; ++c) {
                if (c < nc) {
                    double x[V];
                    unpack<Q>(r, c, m, ragged, x);
#pragma unroll
                    for (int e = 0; e < V; ++e) s = fma(x[e], vl[col[c] + e], s);
                }
            }
            t[r] = wave_sum_f64(s);
        }
        if (wpr > 1) {
            const int wave = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0)
#pragma unroll
                for (int r = 0; r < R; ++r) sh.red[slot][r][wave] = t[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double a = 0.0;
                for (int w = 0; w < wpr; ++w) a += sh.red[slot][r][grp * wpr + w];
                t[r] = a;
            }
            slot ^= 1;
        }
    }

    // The batch's total held by lane r (r < R) of each wave.
    __device__ __forceinline__ double lane_total(const double* t) const {
        const int lane = threadIdx.x & 63;
        double tl = t[0];
#pragma unroll
        for (int r = 1; r < R; ++r)
            if (lane == r) tl = t[r];
        return tl;
    }

    // One batch of an iteration: row totals, the R factors side by side,
    // column accumulation.  The next batch is requested first.
    template <int Q>
    __device__ __forceinline__ void sweep_batch(const BatchDesc& P, int64_t b, const double* vl, int m, bool ragged,
                                                BatchShared& sh, int& slot, uint32_t& fl) {
        load_batch<Q ^ 1>(b + 1);
        double t[R];
        batch_totals<Q>(vl, m, ragged, sh, slot, t);
        const int lane = threadIdx.x & 63;
        const double tl = lane_total(t) * P.k_scale;
        const int64_t il = grp + (int64_t)rg * (b * R + (lane < R ? lane : 0));
        double ul = 0.0;
        if (lane < R && il < P.n) {
            const double ai = abuf[Q];
            ul = batch_factor(ai, tl, P.fi, P.fi_is_one);
            if (gl < R) {              // the group's first wave writes
                P.u[il] = ul;
                if (ai > 0.0 && !(tl > 0.0)) fl |= UOT_FLAG_ZERO_SUM;
                if (!isfinite(ul)) fl |= UOT_FLAG_NONFINITE;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double ur = readlane_f64(ul, r);
#pragma unroll
            for (int c = 0; c < NCM; ++c) {
                if (c < nc) {
                    double x[V];
                    unpack_again<Q>(r, c, m, ragged, x);
#pragma unroll
                    for (int e = 0; e < V; ++e) acc[c * V + e] = fma(x[e], ur, acc[c * V + e]);
                }
            }
        }
    }

    // One batch of the final sweep: r_i = u_i (K v)_i and the objective's row terms.
    template <int Q>
    __device__ __forceinline__ void marg_batch(const BatchDesc& P, int64_t b, const double* vl, int m, bool ragged,
                                               BatchShared& sh, int& slot, double& rlu, double& rsum, double& klr) {
        load_batch<Q ^ 1>(b + 1);
        double t[R];
        batch_totals<Q>(vl, m, ragged, sh, slot, t);
        const int lane = threadIdx.x & 63;
        const double tl = lane_total(t) * P.k_scale;
        const int64_t il = grp + (int64_t)rg * (b * R + (lane < R ? lane : 0));
        if (lane < R && gl < R && il < P.n) {
            const double ui = P.u[il];
            const double ri = ui * tl;
            P.r[il] = ri;
            if (ri > 0.0) rlu += ri * log(ui);
            rsum += ri;
            klr += kl_term(ri, P.a[il]);
        }
    }

    __device__ void run(const BatchDesc& P, const BatchLaunch& B, double* vl, double* wl, BatchShared& sh) {
        const int tid = threadIdx.x;
        const BatchShapeDef sd = kBatchShapes[P.shape];
        rg = sd.rg;
        nc = sd.nc;
        lr = kBatchWG / rg;
        wpr = lr / 64;
        grp = tid / lr;
        gl = tid % lr;
        const int64_t n = P.n;
        const int m = (int)P.m;
        pa = P.a;
        pn = n;
        row_bytes = (uint32_t)(P.ldk * (int64_t)sizeof(KT));
        const uint32_t total = (uint32_t)(n * row_bytes);
        const uint64_t kp = (uint64_t)(uintptr_t)P.K;
        const uint32_t k_lo = __builtin_amdgcn_readfirstlane((uint32_t)kp);
        const uint32_t k_hi = __builtin_amdgcn_readfirstlane((uint32_t)(kp >> 32));
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(((uint64_t)k_hi << 32) | k_lo), (short)0,
                                                 (int)__builtin_amdgcn_readfirstlane(total), kBufferWord3);
#pragma unroll
        for (int c = 0; c < NCM; ++c) {
            col[c] = (c * lr + gl) * V;
            voff[c] = (c < nc && col[c] < m) ? (uint32_t)col[c] * (uint32_t)sizeof(KT) : total;
        }
        const int mpad = nc * lr * V;
        for (int j = tid; j < mpad; j += kBatchWG) vl[j] = (j < m) ? 1.0 : 0.0;
        const double tol = B.tol;
        // Split problem: the parts' column sums (by iteration parity), this
        // part's own copy of the column marginal, the objective row terms.
        const bool split = P.parts > 1;
        const int parts = split ? P.parts : 1;
        const int64_t mx = (m + 1) / 2 * 2;
        uint32_t* hdr = split ? (uint32_t*)(B.pool + kBatchHeaderBytes * (size_t)P.split) : nullptr;
        double* xw = split ? (double*)(B.pool + P.xch) : nullptr;
        double* cm = split ? xw + 2 * parts * mx + P.part * mx : P.c;     // previous column marginal
        double* xo = split ? xw + 3 * parts * mx : nullptr;
        // previous column marginal of the stopping test: c_0 = 0
        if (tol > 0.0)
            for (int j = tid; j < m; j += kBatchWG) cm[j] = 0.0;
        if (tid == 0) sh.flags = 0u;
        __syncthreads();

        const bool ragged = (m % V) != 0;
        uint32_t fl = 0;
        // rows of a group: i = grp + rg k, k < kmax (the same count for every
        // group: groups that exchange row totals step together)
        const int64_t kmax = (n + rg - 1) / rg;
        const int64_t nbatch = (kmax + R - 1) / R;
        int slot = 0;
        int64_t it = 0;
        double err = 0.0;
        bool stopped = false;
        for (int64_t t = 1; t <= B.max_iter; ++t) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0.0;
            load_batch<0>(0);
            for (int64_t bb = 0; bb < nbatch; bb += 2) {
                sweep_batch<0>(P, bb, vl, m, ragged, sh, slot, fl);
                if (bb + 1 < nbatch) sweep_batch<1>(P, bb + 1, vl, m, ragged, sh, slot, fl);
            }
            // Column sums: the groups' partials added in group order.
            if (rg > 1) {
                for (int g = 0; g < rg; ++g) {
                    if (grp == g) {
#pragma unroll
                        for (int c = 0; c < NCM; ++c)
#pragma unroll
                            for (int e = 0; e < V; ++e) {
                                const int j = col[c] + e;
                                if (c < nc && j < m) wl[j] = (g == 0) ? acc[c * V + e] : wl[j] + acc[c * V + e];
                            }
                    }
                    __syncthreads();
                }
            } else {
                __syncthreads();     // every row's use of v is complete
            }
            // Split problem: publish this part's column sums, wait for the
            // other parts; every part then adds all parts' sums in part order
            // into wl.
            if (split) {
                double* xt = xw + (t & 1) * parts * mx;
                if (grp == 0) {
#pragma unroll
                    for (int c = 0; c < NCM; ++c)
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            const int j = col[c] + e;
                            if (c < nc && j < m) xt[P.part * mx + j] = (rg > 1) ? wl[j] : acc[c * V + e];
                        }
                }
                part_barrier(hdr, (uint32_t)(parts * t));
                for (int j = tid; j < m; j += kBatchWG) {
                    double ws = 0.0;
                    for (int q = 0; q < parts; ++q) ws += xt[q * mx + j];
                    wl[j] = ws;
                }
                __syncthreads();
            }
            // Column half-step (group 0 owns each column once), marginal c = v w.
            double dsum = 0.0, csum = 0.0;
            if (grp == 0) {
#pragma unroll
                for (int c = 0; c < NCM; ++c)
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const int j = col[c] + e;
                        if (c < nc && j < m) {
                            const double w = ((rg > 1 || split) ? wl[j] : acc[c * V + e]) * P.k_scale;
                            const double bj = P.b[j];
                            const double vj = batch_factor(bj, w, P.fi, P.fi_is_one);
                            if (bj > 0.0 && !(w > 0.0)) fl |= UOT_FLAG_ZERO_SUM;
                            if (!isfinite(vj)) fl |= UOT_FLAG_NONFINITE;
                            vl[j] = vj;
                            const double cj = vj * w;
                            if (tol > 0.0) {
                                dsum += fabs(cj - cm[j]);
                                csum += fabs(cj);
                            }
                            cm[j] = cj;
                            if (P.part == 0) {
                                P.v[j] = vj;
                                if (split) P.c[j] = cj;
                            }
                        }
                    }
            }
            it = t;
            if (tol > 0.0 && (t % B.check_every) == 0) {
                const double ds = block_sum(dsum, sh.scratch);
                const double cs = block_sum(csum, sh.scratch);
                err = ds / cs;
                if (err <= tol) stopped = true;
            }
            __syncthreads();     // v complete in LDS before the next sweep
            if (stopped) break;
        }

        // Row marginal r = u (K v) with the final v, and the objective's terms.
        double rlu = 0.0, rsum = 0.0, klr = 0.0;
        load_batch<0>(0);
        for (int64_t bb = 0; bb < nbatch; bb += 2) {
            marg_batch<0>(P, bb, vl, m, ragged, sh, slot, rlu, rsum, klr);
            if (bb + 1 < nbatch) marg_batch<1>(P, bb + 1, vl, m, ragged, sh, slot, rlu, rsum, klr);
        }
        double clv = 0.0, klc = 0.0;
        if (grp == 0) {
#pragma unroll
            for (int c = 0; c < NCM; ++c)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = col[c] + e;
                    if (c < nc && j < m) {
                        const double cj = cm[j];
                        if (cj > 0.0) clv += cj * log(vl[j]);
                        klc += kl_term(cj, P.b[j]);
                    }
                }
        }
        if (fl) atomicOr(&sh.flags, fl);
        double s_rlu = block_sum(rlu, sh.scratch);
        double s_r = block_sum(rsum, sh.scratch);
        const double s_clv = block_sum(clv, sh.scratch);
        double s_klr = block_sum(klr, sh.scratch);
        const double s_klc = block_sum(klc, sh.scratch);
        uint32_t part_flags = 0u;
        if (split) {
            // row terms of all parts, added in part order by part 0
            if (tid == 0) {
                xo[4 * P.part] = s_rlu;
                xo[4 * P.part + 1] = s_r;
                xo[4 * P.part + 2] = s_klr;
                if (sh.flags) atomicOr(&hdr[1], sh.flags);
            }
            part_barrier(hdr, (uint32_t)(parts * (it + 1)));
            if (P.part != 0) return;
            s_rlu = s_r = s_klr = 0.0;
            for (int q = 0; q < parts; ++q) {
                s_rlu += xo[4 * q];
                s_r += xo[4 * q + 1];
                s_klr += xo[4 * q + 2];
            }
            part_flags = __hip_atomic_load(&hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        double L = P.eps * (s_rlu + s_clv - s_r);
        if (!P.fi_is_one) L += P.tau * (s_klr + s_klc);
        if (tid == 0) {
            *P.loss = L;
            uint32_t flags = sh.flags | part_flags;
            if (!isfinite(L)) flags |= UOT_FLAG_NONFINITE;
            if (tol > 0.0 && !stopped) flags |= UOT_FLAG_NOT_CONVERGED;
            P.info->iters = it;
            P.info->err = err;
            P.info->absorptions = 0;
            P.info->flags = flags;
        }
        __syncthreads();
    }
};

template <typename KT>
__global__ __launch_bounds__(kBatchWG, 2) void batch_kernel(BatchLaunch B) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BatchShared sh;
    double* vl = (double*)smem;
    double* wl = vl + B.m_lds;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const int32_t idx = (int32_t)atomicAdd(B.next, 1u);
            sh.idx = idx;
            if (B.trace && idx < B.count) B.trace[2 * idx] = wall_clock64();
        }
        __syncthreads();
        const int32_t idx = __builtin_amdgcn_readfirstlane(sh.idx);   // uniform: descriptor in SGPRs
        __syncthreads();
        if (idx >= B.count) break;
        const BatchDesc P = B.desc[idx];
        BatchSolve<KT> s;
        s.run(P, B, vl, wl, sh);
        if (tid == 0 && B.trace) B.trace[2 * idx + 1] = wall_clock64();
    }
}

// Queue head and the split problems' counters and flags to 0.
__global__ void batch_reset_kernel(uint32_t* next, uint32_t* headers, int32_t words) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *next = 0u;
    for (int32_t w = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); w < words; w += gridDim.x * blockDim.x)
        headers[w] = 0u;
}

template <typename KT>
const void* batch_fn() {
    return (const void*)batch_kernel<KT>;
}

const void* batch_lookup(int k_dtype) {
    switch (k_dtype) {
        case UOT_F64: return batch_fn<double>();
        case UOT_F32: return batch_fn<float>();
        case UOT_BF16: return batch_fn<bf16_t>();
        case UOT_FP8_E4M3: return batch_fn<fp8_t>();
        default: return nullptr;
    }
}

int elem_bytes_of(int k_dtype) {
    switch (k_dtype) {
        case UOT_F64: return 8;
        case UOT_F32: return 4;
        case UOT_BF16: return 2;
        default: return 1;
    }
}

}  // namespace

int batch_shape_count() { return kNumBatchShapes; }

bool batch_shape_ok(int shape, int k_dtype) {
    if (shape < 0 || shape >= kNumBatchShapes) return false;
    const int v = 16 / elem_bytes_of(k_dtype);
    const int ncm = v >= kLaneCols ? 1 : kLaneCols / v;
    return kBatchShapes[shape].nc <= ncm;
}

// Columns a shape covers for a stored type.
int64_t batch_shape_max_m(int shape, int k_dtype) {
    const BatchShapeDef d = kBatchShapes[shape];
    return (int64_t)d.nc * (kBatchWG / d.rg) * (16 / elem_bytes_of(k_dtype));
}

int batch_shape_rows(int shape) { return kBatchShapes[shape].rg; }
int batch_shape_chunks(int shape) { return kBatchShapes[shape].nc; }

size_t batch_lds_bytes(int64_t m_lds) { return sizeof(double) * 2 * (size_t)m_lds; }

int batch_max_grid(int k_dtype, size_t lds) {
    const void* fn = batch_lookup(k_dtype);
    if (!fn) return 0;
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchWG, lds) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_batch(int k_dtype, const BatchLaunch& B, int grid, size_t lds, hipStream_t stream) {
    const void* fn = batch_lookup(k_dtype);
    if (!fn) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int32_t hwords = (int32_t)(B.nsplit * kBatchHeaderBytes / sizeof(uint32_t));
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, stream, B.next, (uint32_t*)B.pool, hwords);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&B};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBatchWG), args, lds, stream);
}

}  // namespace uot
