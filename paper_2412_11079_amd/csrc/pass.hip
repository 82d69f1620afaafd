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
// (chunk c of lane t starts at column (c*WG + t)*V), so one wave's load of a
// chunk is 1 KiB of contiguous HBM.  Rows are software-pipelined D deep:
// while row i is reduced (one barrier per row) and accumulated, the loads of
// rows i+1 .. i+D-1 are in flight in registers.  K is read through a buffer
// resource spanning the workgroup's strip, so the prefetch past the strip's
// last row and the chunks of lanes beyond column m read as zeros without a
// branch.  Per-row inputs (a, or u) are staged in LDS before the loop so
// that no global load is waited on between prefetch and use.
#include "uot_common.h"

namespace uot {

// Word 3 of a raw buffer resource on gfx9-class parts (untyped 32-bit data).
constexpr int kBufferWord3 = 0x00020000;
// Cache policy of the K loads (0: default).
#ifndef UOT_K_LOAD_AUX
#define UOT_K_LOAD_AUX 0
#endif
constexpr int kLoadAux = UOT_K_LOAD_AUX;

template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int MODE>
__global__ __launch_bounds__(WG) void pass_kernel(PassLaunch L) {
    using KV = KVec<KT>;
    using Raw = typename KV::raw;
    constexpr int V = KV::N;
    constexpr int E = NC * V;
    constexpr int NW = WG / 64;
    constexpr bool kDot = (MODE != MODE_COL);
    constexpr bool kAcc = (MODE != MODE_ROW);
    constexpr bool kVreg = kDot && !VLDS;

    __shared__ double red[2][NW];
    extern __shared__ __align__(16) unsigned char dyn_lds[];

    if (L.check_done && ld_volatile_u32(&L.ctrl->done)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t m = L.m;
    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);

    // LDS: [v as AT, padded to ldv] [row input: a or u] [row shift]
    AT* vl = (AT*)dyn_lds;
    double* row_in = (double*)(dyn_lds + (VLDS && kDot ? L.ldv_bytes : 0));
    double* row_sh = row_in + L.rows_per_wg;
    for (int k = tid; k < nrows; k += WG) {
        if constexpr (MODE == MODE_FUSED || MODE == MODE_ROW) {
            row_in[k] = L.a[r0 + k];
            row_sh[k] = L.fpot ? -(1.0 - L.fi) * L.fpot[r0 + k] * L.inv_eps : 0.0;
        } else {
            row_in[k] = L.u[r0 + k];
        }
    }
    if constexpr (VLDS && kDot) {
        const int64_t mv = (m + V - 1) / V * V;
        for (int64_t j = tid; j < mv; j += WG) vl[j] = (j < m) ? (AT)L.v[j] : (AT)0;
    }
    __syncthreads();

    // Buffer resource over this workgroup's strip of rows.
    const uint32_t row_bytes = (uint32_t)(L.ldk * (int64_t)sizeof(KT));
    const uint32_t strip_bytes = (uint32_t)((int64_t)nrows * L.ldk * (int64_t)sizeof(KT));
    const KT* strip = (const KT*)L.K + r0 * L.ldk;
    __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)strip, (short)0, (int)strip_bytes, kBufferWord3);

    int64_t col[NC];
    uint32_t voff[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        col[c] = ((int64_t)c * WG + tid) * V;
        voff[c] = col[c] < m ? (uint32_t)(col[c] * (int64_t)sizeof(KT)) : strip_bytes;
    }
    const bool ragged = (m % V) != 0;

    AT vv[kVreg ? E : 1];
    if constexpr (kVreg) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                int64_t j = col[c] + e;
                vv[c * V + e] = (j < m) ? (AT)L.v[j] : (AT)0;
            }
    }
    AT acc[kAcc ? E : 1];
#pragma unroll
    for (int e = 0; e < (kAcc ? E : 1); ++e) acc[e] = (AT)0;

    Raw buf[D][NC];

    auto load_row = [&](Raw (&b)[NC], int k) {
        // k = row index within the strip; rows >= nrows land past strip_bytes (zeros)
        const uint32_t soff = (uint32_t)k * row_bytes;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            b[c] = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)voff[c], (int)soff,
                                                                                 kLoadAux));
    };

    int slot = 0;
    auto process = [&](Raw (&b)[NC], int k) {
        AT ur;
        if constexpr (kDot) {
            AT s = (AT)0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                AT x[V];
                unpack<AT>(b[c], x);
                if (ragged) {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (col[c] + e >= m) x[e] = (AT)0;
                }
                if constexpr (VLDS) {
                    if (col[c] < m) {
#pragma unroll
                        for (int e = 0; e < V; ++e) s = fma(x[e], vl[col[c] + e], s);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e) s = fma(x[e], vv[c * V + e], s);
                }
            }
            double d = wave_sum_f64((double)s);
            if (lane == 0) red[slot][wave] = d;
            __syncthreads();
            // Every lane forms the row total in the same fixed order.
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tot += red[slot][w];
            slot ^= 1;
            double uval;
            if constexpr (MODE == MODE_MARG) {
                uval = row_in[k];
                if (tid == 0) L.s_out[r0 + k] = tot;
            } else {
                const double ai = row_in[k];
                uval = scale_factor(ai, tot, L.fi, L.fi_is_one, row_sh[k]);
                if (tid == 0) {
                    L.u[r0 + k] = uval;
                    if (ai > 0.0 && !(tot > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
                    if (!isfinite(uval)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
                }
            }
            ur = (AT)uval;
        } else {
            ur = (AT)row_in[k];
        }
        if constexpr (kAcc) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                AT x[V];
                unpack<AT>(b[c], x);
#pragma unroll
                for (int e = 0; e < V; ++e) acc[c * V + e] = fma(x[e], ur, acc[c * V + e]);
            }
        }
    };

    // Prologue: rows 0 .. D-2 in flight.
#pragma unroll
    for (int q = 0; q < D - 1; ++q) load_row(buf[q], q);
    for (int k0 = 0; k0 < nrows; k0 += D) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int k = k0 + q;
            if (k >= nrows) break;
            load_row(buf[(q + D - 1) % D], k + D - 1);
            process(buf[q], k);
        }
    }

    if constexpr (kAcc) {
        AT* P = (AT*)L.partials + (int64_t)blockIdx.x * L.ldp;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (col[c] >= m) continue;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                // ldp is a multiple of 64 >= m, so the whole chunk lies inside the partial row.
                P[col[c] + e] = acc[c * V + e];
            }
        }
    }
}

// Instantiated launch shapes {WG, NC, D, v in LDS}.
static const PassShape kShapes[] = {
    {256, 1, 4, 0},    // 0: short rows
    {512, 1, 4, 0},    // 1
    {1024, 1, 4, 0},   // 2
    {1024, 2, 3, 0},   // 3
    {512, 4, 3, 0},    // 4
    {512, 8, 2, 1},    // 5: 16384 FP32 columns, 8 waves, v in LDS
    {1024, 4, 2, 1},   // 6: 16384 FP32 columns, 16 waves, v in LDS
    {512, 8, 3, 1},    // 7: as 5, three rows in flight
};
static constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int pass_shape_count() { return kNumShapes; }
PassShape pass_shape(int idx) { return kShapes[idx]; }

// Launch one instantiation; raises its dynamic-LDS limit first when the
// request exceeds the default 64 KiB (once per size increase).
template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int MODE>
static hipError_t launch_one(const PassLaunch& L, size_t lds, hipStream_t stream) {
    static size_t raised = 65536;
    auto fn = pass_kernel<KT, AT, WG, NC, D, VLDS, MODE>;
    if (lds > raised) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        raised = lds;
    }
    hipLaunchKernelGGL(fn, dim3(L.grid), dim3(WG), lds, stream, L);
    return hipGetLastError();
}

template <typename KT, typename AT, int WG, int NC, int D, bool VLDS>
static hipError_t launch_shape(int mode, const PassLaunch& L, size_t lds, hipStream_t stream) {
    switch (mode) {
        case MODE_FUSED: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_FUSED>(L, lds, stream);
        case MODE_ROW: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_ROW>(L, lds, stream);
        case MODE_COL: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_COL>(L, lds, stream);
        case MODE_MARG: return launch_one<KT, AT, WG, NC, D, VLDS, MODE_MARG>(L, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename KT, typename AT>
static hipError_t launch_typed(int mode, int shape_idx, const PassLaunch& L, size_t lds, hipStream_t stream) {
    switch (shape_idx) {
        case 0: return launch_shape<KT, AT, 256, 1, 4, false>(mode, L, lds, stream);
        case 1: return launch_shape<KT, AT, 512, 1, 4, false>(mode, L, lds, stream);
        case 2: return launch_shape<KT, AT, 1024, 1, 4, false>(mode, L, lds, stream);
        case 3: return launch_shape<KT, AT, 1024, 2, 3, false>(mode, L, lds, stream);
        case 4: return launch_shape<KT, AT, 512, 4, 3, false>(mode, L, lds, stream);
        case 5: return launch_shape<KT, AT, 512, 8, 2, true>(mode, L, lds, stream);
        case 6: return launch_shape<KT, AT, 1024, 4, 2, true>(mode, L, lds, stream);
        case 7: return launch_shape<KT, AT, 512, 8, 3, true>(mode, L, lds, stream);
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

hipError_t launch_pass(int k_dtype, int acc64, int mode, int shape_idx, const PassLaunch& L,
                       hipStream_t stream) {
    size_t lds = pass_lds_bytes(shape_idx, mode, acc64, L);
    if (k_dtype == UOT_F64) return launch_typed<double, double>(mode, shape_idx, L, lds, stream);
    if (k_dtype == UOT_F32) {
        if (acc64) return launch_typed<float, double>(mode, shape_idx, L, lds, stream);
        return launch_typed<float, float>(mode, shape_idx, L, lds, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace uot
