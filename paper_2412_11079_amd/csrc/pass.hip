// Streaming passes over K (row half-step, column half-step, or both fused).
//
// Paper Section 4: each iteration is split into four parts; parts 2 and 4
// (rescaling with accumulation of the opposite sums) are the O(nm) work and
// the paper interleaves them so each row is touched once per iteration
// (Section 4.1's single double loop, Algorithm 1's per-thread column
// partials reduced at the end).  Here K is read-only and the scalings are
// vectors, so the fused pass reads each K row exactly once:
//
//   for each row i of this workgroup's strip:
//       s_i = sum_j K_ij v_j                (lane FMAs, wave64 + LDS reduce, FP64)
//       u_i = (a_i / s_i)^fi                (in-kernel, FP64)
//       p_j += K_ij u_i                     (register-resident column partials)
//   write p to the strip's partial row       (deterministic; no atomics)
//
// Workgroup shape: WG lanes each own NC 16-byte column chunks of every row
// (chunk c of lane l in wave w is chunk (w*NC + c)*64 + l), so one wave's
// load of a chunk is 1 KiB of contiguous HBM and its NC loads one block.  Rows are software-pipelined D deep:
// while row i is reduced (one barrier per row) and accumulated, the loads of
// rows i+1 .. i+D-1 are in flight in registers.  K is read through a buffer
// resource spanning the workgroup's strip, so the prefetch past the strip's
// last row and the chunks of lanes beyond column m read as zeros without a
// branch.  Per-row inputs (a, or u) are staged in LDS before the loop so
// that no global load is waited on between prefetch and use.
#include <mutex>

#include "strip.h"

namespace uot {

// ---------------------------------------------------------------------------
// Per-iteration pass kernel.
// ---------------------------------------------------------------------------
template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int MODE, int RB>
__global__ __launch_bounds__(WG) void pass_kernel(PassLaunch L) {
    using S = Strip<KT, AT, WG, NC, D, VLDS, MODE, RB>;
    __shared__ double red[2][S::NW * RB];
    __shared__ uint32_t exit_sh;
    extern __shared__ __align__(16) unsigned char dyn_lds[];

    if (pass_exit(L, &exit_sh)) return;

    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);

    S st;
    st.setup(L, r0, nrows);
    st.prime();

    // LDS: [v as AT, padded to ldv] [row input: a or u] [row shift]
    AT* vl = (AT*)dyn_lds;
    double* row_in = (double*)(dyn_lds + (VLDS && S::kDot ? L.ldv_bytes : 0));
    double* row_sh = row_in + L.rows_per_wg;
    stage_rows<S, MODE, VLDS, AT>(L, r0, nrows, row_in, row_sh);
    if constexpr (VLDS && S::kDot) stage_v<S::V, WG, AT>(L.v, L.m, vl);
    __syncthreads();
    st.load_v_regs(L.v);
    st.clear_acc();
    st.stream(L, vl, row_in, row_sh, red);
    st.store_partials((AT*)L.partials + (int64_t)blockIdx.x * L.ldp);
}

// ---------------------------------------------------------------------------
// Persistent kernel: the whole iteration loop in one cooperative launch.
// Per iteration: fused pass over the strip, grid barrier, column finalize of
// this workgroup's column block (the same fixed-order FP64 sums as the
// finalize kernel), grid barrier.  The launch must be co-resident (checked
// by the cooperative launch); every barrier wait is bounded.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void grid_barrier(uint32_t* count, uint32_t target, uint32_t* flags) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(count, 1u);
        uint32_t spins = 0;
        while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kBarrierSpinLimit) {
                atomicOr(flags, UOT_FLAG_BARRIER_TIMEOUT);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename KT, typename AT, int WG, int NC, int D, bool VLDS>
__global__ __launch_bounds__(WG) void persist_kernel(PersistLaunch P) {
    using S = Strip<KT, AT, WG, NC, D, VLDS, MODE_FUSED>;
    __shared__ double red[2][S::NW];
    __shared__ double err_sh;
    __shared__ double fin_red[2][S::NW];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const PassLaunch& L = P.L;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint32_t G = gridDim.x;

    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);

    // LDS: [v / finalize scratch (max of both)] [a strip] [shift strip]
    AT* vl = (AT*)dyn_lds;
    double* fin = (double*)dyn_lds;
    double* row_in = (double*)(dyn_lds + P.scratch_bytes);
    double* row_sh = row_in + L.rows_per_wg;
    stage_rows<S, MODE_FUSED, VLDS, AT>(L, r0, nrows, row_in, row_sh);

    // Column block finalized by this workgroup: [cb0, cb0 + P.fin_cols).
    const int64_t cb0 = (int64_t)blockIdx.x * P.fin_cols;
    const int groups = P.fin_cols / 4;            // 4-column chunks
    const int phases = WG / groups;               // strip phases per chunk
    const int cg = tid % groups;
    const int ph = tid / groups;

    S st;
    st.setup(L, r0, nrows);
    uint32_t bar = 0;
    int64_t t = 1;
    for (; t <= P.max_iter; ++t) {
        if (stop_test(L, t, &err_sh)) break;
        st.prime();
        if constexpr (VLDS) stage_v<S::V, WG, AT>(L.v, L.m, vl);
        __syncthreads();
        st.load_v_regs(L.v);
        st.clear_acc();
        st.stream(L, vl, row_in, row_sh, red);
        st.store_partials((AT*)L.partials + (int64_t)blockIdx.x * L.ldp);
        bar += G;
        grid_barrier(&L.ctrl->bar, bar, &L.ctrl->flags);

        // ---- column finalize of this workgroup's block
        double accf[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t c0 = cb0 + 4 * cg;
        if (ph < phases && c0 < L.m) {
            const AT* Pp = (const AT*)L.partials + c0;
            for (int g = ph; g < (int)G; g += phases) {
                double x[4];
                Chunk4<AT>::load(Pp + (int64_t)g * L.ldp, x);
#pragma unroll
                for (int e = 0; e < 4; ++e) accf[e] += x[e];
            }
        }
        __syncthreads();   // v in LDS is dead from here; reuse it as scratch
        if (ph < phases) {
#pragma unroll
            for (int e = 0; e < 4; ++e) fin[ph * P.fin_cols + 4 * cg + e] = accf[e];
        }
        __syncthreads();
        double dsum = 0.0, csum = 0.0;
        if (tid < P.fin_cols) {
            const int64_t j = cb0 + tid;
            double w = 0.0;
            for (int q = 0; q < phases; ++q) w += fin[q * P.fin_cols + tid];
            w *= P.F.k_scale;
            if (j < L.m) {
                const FinLaunch& F = P.F;
                const double bj = F.b[j];
                double shift = F.gpot ? -(1.0 - F.fi) * F.gpot[j] * F.inv_eps : 0.0;
                double vj = scale_factor(bj, w, F.fi, F.fi_is_one, shift);
                F.v[j] = vj;
                F.w_out[j] = w;
                double cj = vj * w;
                double cp = F.cprev[j];
                F.cprev[j] = cj;
                dsum = fabs(cj - cp);
                csum = fabs(cj);
                if (bj > 0.0 && !(w > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
                if (!isfinite(vj)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
            }
        }
        // block sums for the stopping test, in a fixed order
        if (tid < ((P.fin_cols + 63) & ~63)) {
            dsum = wave_sum_f64(dsum);
            csum = wave_sum_f64(csum);
            if (lane == 0) {
                fin_red[0][wave] = dsum;
                fin_red[1][wave] = csum;
            }
        }
        __syncthreads();
        if (tid == 0) {
            double a0 = 0.0, a1 = 0.0;
            for (int w = 0; w < (P.fin_cols + 63) / 64; ++w) {
                a0 += fin_red[0][w];
                a1 += fin_red[1][w];
            }
            P.F.blockpart[2 * blockIdx.x] = a0;
            P.F.blockpart[2 * blockIdx.x + 1] = a1;
        }
        bar += G;
        grid_barrier(&L.ctrl->bar, bar, &L.ctrl->flags);
    }
}

// Instantiated launch shapes {WG, NC, D, v in LDS, rows per barrier}.
static const PassShape kShapes[] = {
    {256, 1, 4, 0, 1},    // 0: short rows
    {512, 1, 4, 0, 1},    // 1
    {1024, 1, 4, 0, 1},   // 2
    {1024, 2, 3, 0, 1},   // 3
    {512, 4, 3, 0, 1},    // 4
    {512, 8, 2, 1, 1},    // 5: 16384 FP32 columns, 8 waves, v in LDS
    {1024, 4, 2, 1, 1},   // 6: 16384 FP32 columns, 16 waves, v in LDS
    {512, 8, 3, 1, 1},    // 7: as 5, three rows in flight
    {1024, 2, 2, 0, 2},   // 8: 8192 FP32 columns, batches of 2 rows
    {1024, 1, 2, 0, 4},   // 9: 4096 FP32 / 8192 BF16 columns, batches of 4 rows
    {512, 1, 2, 0, 4},    // 10: 2048 FP32 / 8192 FP8 columns, batches of 4 rows
    {256, 1, 2, 0, 4},    // 11: 1024 FP32 columns, batches of 4 rows
    {512, 4, 2, 0, 2},    // 12: 8192 FP32 columns, 512 lanes, batches of 2 rows
    {512, 2, 2, 0, 4},    // 13: 8192 BF16 columns, 512 lanes, batches of 4 rows
    {512, 1, 2, 0, 8},    // 14: 8192 FP8 columns, 512 lanes, batches of 8 rows
};
static constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int pass_shape_count() { return kNumShapes; }
PassShape pass_shape(int idx) { return kShapes[idx]; }

// Launch one instantiation; raises its dynamic-LDS limit first when the
// request exceeds the default 64 KiB (once per device and size increase; the
// attribute belongs to the device the call runs on).
// With `resident` set, nothing is launched: *resident receives how many
// workgroups of this instantiation fit on one CU with `lds` bytes of LDS.
template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int MODE, int RB>
static hipError_t launch_one(const PassLaunch& L, size_t lds, hipStream_t stream, int* resident) {
    constexpr int kDevs = 64;
    static std::mutex mu;
    static size_t raised[kDevs];
    auto fn = pass_kernel<KT, AT, WG, NC, D, VLDS, MODE, RB>;
    if (lds > 65536) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        bool need = true;
        if (dev >= 0 && dev < kDevs) {
            std::lock_guard<std::mutex> lk(mu);
            need = lds > raised[dev];
        }
        if (need) {
            e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            if (dev >= 0 && dev < kDevs) {
                std::lock_guard<std::mutex> lk(mu);
                if (lds > raised[dev]) raised[dev] = lds;
            }
        }
    }
    if (resident) return hipOccupancyMaxActiveBlocksPerMultiprocessor(resident, (const void*)fn, WG, lds);
    hipLaunchKernelGGL(fn, dim3(L.grid), dim3(WG), lds, stream, L);
    return hipGetLastError();
}

template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int RB = 1>
static hipError_t launch_shape(int mode, const PassLaunch& L, size_t lds, hipStream_t stream, int* resident) {
    switch (mode) {
        case MODE_FUSED: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_FUSED, RB>(L, lds, stream, resident);
        case MODE_ROW: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_ROW, RB>(L, lds, stream, resident);
        case MODE_COL: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_COL, RB>(L, lds, stream, resident);
        case MODE_MARG: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_MARG, RB>(L, lds, stream, resident);
        default: return hipErrorInvalidValue;
    }
}

template <typename KT, typename AT>
static hipError_t launch_typed(int mode, int shape_idx, const PassLaunch& L, size_t lds, hipStream_t stream,
                               int* resident) {
    switch (shape_idx) {
        case 0: return launch_shape<KT, AT, 256, 1, 4, false>(mode, L, lds, stream, resident);
        case 1: return launch_shape<KT, AT, 512, 1, 4, false>(mode, L, lds, stream, resident);
        case 2: return launch_shape<KT, AT, 1024, 1, 4, false>(mode, L, lds, stream, resident);
        case 3: return launch_shape<KT, AT, 1024, 2, 3, false>(mode, L, lds, stream, resident);
        case 4: return launch_shape<KT, AT, 512, 4, 3, false>(mode, L, lds, stream, resident);
        case 5: return launch_shape<KT, AT, 512, 8, 2, true>(mode, L, lds, stream, resident);
        case 6: return launch_shape<KT, AT, 1024, 4, 2, true>(mode, L, lds, stream, resident);
        case 7: return launch_shape<KT, AT, 512, 8, 3, true>(mode, L, lds, stream, resident);
        case 8: return launch_shape<KT, AT, 1024, 2, 2, false, 2>(mode, L, lds, stream, resident);
        case 9: return launch_shape<KT, AT, 1024, 1, 2, false, 4>(mode, L, lds, stream, resident);
        case 10: return launch_shape<KT, AT, 512, 1, 2, false, 4>(mode, L, lds, stream, resident);
        case 11: return launch_shape<KT, AT, 256, 1, 2, false, 4>(mode, L, lds, stream, resident);
        case 12: return launch_shape<KT, AT, 512, 4, 2, false, 2>(mode, L, lds, stream, resident);
        case 13: return launch_shape<KT, AT, 512, 2, 2, false, 4>(mode, L, lds, stream, resident);
        case 14: return launch_shape<KT, AT, 512, 1, 2, false, 8>(mode, L, lds, stream, resident);
        default: return hipErrorInvalidValue;
    }
}

// The in-place matrix form: one-row shapes (0-7), storage type = lane type.
template <typename KT>
static hipError_t launch_matrix_typed(int shape_idx, const PassLaunch& L, size_t lds, hipStream_t stream) {
    switch (shape_idx) {
        case 0: return launch_one<KT, KT, 256, 1, 4, false, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 1: return launch_one<KT, KT, 512, 1, 4, false, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 2: return launch_one<KT, KT, 1024, 1, 4, false, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 3: return launch_one<KT, KT, 1024, 2, 3, false, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 4: return launch_one<KT, KT, 512, 4, 3, false, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 5: return launch_one<KT, KT, 512, 8, 2, true, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 6: return launch_one<KT, KT, 1024, 4, 2, true, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        case 7: return launch_one<KT, KT, 512, 8, 3, true, MODE_MATRIX, 1>(L, lds, stream, nullptr);
        default: return hipErrorInvalidValue;
    }
}

size_t pass_lds_bytes(int shape_idx, int mode, int acc64, const PassLaunch& L) {
    PassShape s = kShapes[shape_idx];
    size_t b = sizeof(double) * 2 * (size_t)L.rows_per_wg;
    if (s.vlds && mode != MODE_COL) b += (size_t)L.ldv_bytes;
    (void)acc64;
    return b;
}

static hipError_t dispatch_pass(int k_dtype, int acc64, int mode, int shape_idx, const PassLaunch& L, size_t lds,
                                hipStream_t stream, int* resident) {
    if (k_dtype == UOT_F64) return launch_typed<double, double>(mode, shape_idx, L, lds, stream, resident);
    if (k_dtype == UOT_F32) {
        if (acc64) return launch_typed<float, double>(mode, shape_idx, L, lds, stream, resident);
        return launch_typed<float, float>(mode, shape_idx, L, lds, stream, resident);
    }
    if (k_dtype == UOT_BF16) return launch_typed<bf16_t, float>(mode, shape_idx, L, lds, stream, resident);
    if (k_dtype == UOT_FP8_E4M3) return launch_typed<fp8_t, float>(mode, shape_idx, L, lds, stream, resident);
    return hipErrorInvalidValue;
}

hipError_t launch_pass(int k_dtype, int acc64, int mode, int shape_idx, const PassLaunch& L,
                       hipStream_t stream) {
    return dispatch_pass(k_dtype, acc64, mode, shape_idx, L, pass_lds_bytes(shape_idx, mode, acc64, L), stream,
                         nullptr);
}

hipError_t launch_pass_matrix(int k_dtype, int shape_idx, const PassLaunch& L, hipStream_t stream) {
    const size_t lds = pass_lds_bytes(shape_idx, MODE_MATRIX, k_dtype == UOT_F64, L);
    if (k_dtype == UOT_F64) return launch_matrix_typed<double>(shape_idx, L, lds, stream);
    if (k_dtype == UOT_F32) return launch_matrix_typed<float>(shape_idx, L, lds, stream);
    return hipErrorInvalidValue;
}

int pass_resident_per_cu(int k_dtype, int acc64, int mode, int shape_idx, size_t lds) {
    int per_cu = 0;
    PassLaunch L{};
    if (dispatch_pass(k_dtype, acc64, mode, shape_idx, L, lds, nullptr, &per_cu) != hipSuccess) return 0;
    return per_cu;
}


// ---------------------------------------------------------------------------
// Persistent launch
// ---------------------------------------------------------------------------
template <typename KT, typename AT, int WG, int NC, int D, bool VLDS>
static const void* persist_fn() {
    return (const void*)persist_kernel<KT, AT, WG, NC, D, VLDS>;
}

template <typename KT, typename AT>
static const void* persist_typed(int shape_idx, int* wg) {
    switch (shape_idx) {
        case 0: *wg = 256; return persist_fn<KT, AT, 256, 1, 4, false>();
        case 1: *wg = 512; return persist_fn<KT, AT, 512, 1, 4, false>();
        case 2: *wg = 1024; return persist_fn<KT, AT, 1024, 1, 4, false>();
        case 3: *wg = 1024; return persist_fn<KT, AT, 1024, 2, 3, false>();
        case 4: *wg = 512; return persist_fn<KT, AT, 512, 4, 3, false>();
        case 5: *wg = 512; return persist_fn<KT, AT, 512, 8, 2, true>();
        case 6: *wg = 1024; return persist_fn<KT, AT, 1024, 4, 2, true>();
        case 7: *wg = 512; return persist_fn<KT, AT, 512, 8, 3, true>();
        default: return nullptr;
    }
}

static const void* persist_lookup(int k_dtype, int acc64, int shape_idx, int* wg) {
    if (k_dtype == UOT_F64) return persist_typed<double, double>(shape_idx, wg);
    if (k_dtype == UOT_F32) {
        if (acc64) return persist_typed<float, double>(shape_idx, wg);
        return persist_typed<float, float>(shape_idx, wg);
    }
    return nullptr;
}

int persist_max_grid(int k_dtype, int acc64, int shape_idx, size_t lds) {
    int wg = 0;
    const void* fn = persist_lookup(k_dtype, acc64, shape_idx, &wg);
    if (!fn) return 0;
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int dev = 0, cus = 0, coop = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, lds) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_persist(int k_dtype, int acc64, int shape_idx, const PersistLaunch& P, size_t lds,
                          hipStream_t stream) {
    int wg = 0;
    const void* fn = persist_lookup(k_dtype, acc64, shape_idx, &wg);
    if (!fn) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    PersistLaunch arg = P;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3(P.L.grid), dim3(wg), args, (unsigned)lds, stream);
}

}  // namespace uot
