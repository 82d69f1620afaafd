// One workgroup's streaming pass over a strip of rows of K (shared by the
// forward pass kernels and the adjoint pass).
#pragma once

#include "uot_common.h"

namespace uot {

// Word 3 of a raw buffer resource on gfx9-class parts (untyped 32-bit data).
constexpr int kBufferWord3 = 0x00020000;
// Cache-policy bits of the K loads.
// 2 = non-temporal: K is streamed once per pass and should not displace v,
// the partials or other workgroups' lines in L2 / the memory-side cache.
#ifndef UOT_K_LOAD_AUX
#define UOT_K_LOAD_AUX 2
#endif
constexpr int kLoadAux = UOT_K_LOAD_AUX;

// ---------------------------------------------------------------------------
// One workgroup's streaming pass over its strip of rows.  Shared by the
// per-iteration pass kernel and the persistent kernel.
// ---------------------------------------------------------------------------
// RB > 1: rows are taken in batches of RB.  The batch's dot products are
// reduced together (one LDS exchange and one barrier per batch) and its RB
// scaling factors are evaluated side by side, lane r of every wave taking
// row r, then broadcast; for short rows this divides the per-row chain of
// reduction, barrier and FP64 power by RB.  D then counts batches in flight.
template <typename KT, typename AT, int WG, int NC, int D, bool VLDS, int MODE, int RB = 1>
struct Strip {
    using KV = KVec<KT>;
    using Raw = typename KV::raw;
    static constexpr int V = KV::N;
    static constexpr int E = NC * V;
    static constexpr int NW = WG / 64;
    static constexpr bool kDot = (MODE != MODE_COL);
    static constexpr bool kAcc = (MODE != MODE_ROW);
    static constexpr bool kVreg = kDot && !VLDS;

    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t row_bytes;
    int64_t m;
    int64_t r0;
    int nrows;
    bool ragged;
    int64_t col[NC];
    uint32_t voff[NC];
    Raw buf[D * RB][NC];
    AT vv[kVreg ? E : 1];
    AT acc[kAcc ? E : 1];

    __device__ __forceinline__ void setup(const PassLaunch& L, int64_t r0_, int nrows_) {
        m = L.m;
        r0 = r0_;
        nrows = nrows_;
        row_bytes = (uint32_t)(L.ldk * (int64_t)sizeof(KT));
        // Buffer resource over the strip: loads past its last row and the
        // chunks of lanes beyond column m (offset set to the strip size) read 0.
        // The row offset is part of the lane offset, so the range check
        // covers it; the host keeps (rows + 16) row_bytes below 2^31, so the
        // sum never wraps.
        const uint32_t strip_bytes = (uint32_t)((int64_t)nrows * L.ldk * (int64_t)sizeof(KT));
        const KT* strip = (const KT*)L.K + r0 * L.ldk;
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)strip, (short)0, (int)strip_bytes, kBufferWord3);
        // Chunk c of lane l in wave w: chunk (w NC + c) 64 + l of the row, so
        // each load instruction reads 1 KiB and a wave's NC loads one
        // contiguous NC KiB block (measured 3% faster on 16384-column rows
        // than interleaving the waves' chunks at a WG-chunk stride).
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            col[c] = ((int64_t)((threadIdx.x >> 6) * NC + c) * 64 + (threadIdx.x & 63)) * V;
            voff[c] = col[c] < m ? (uint32_t)(col[c] * (int64_t)sizeof(KT)) : strip_bytes;
        }
        ragged = (m % V) != 0;
    }

    template <int Q>
    __device__ __forceinline__ void load_row(int k) {
        const uint32_t soff = (uint32_t)k * row_bytes;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            buf[Q][c] = __builtin_bit_cast(
                Raw, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(voff[c] + soff), 0, kLoadAux));
    }

    // Rows kb RB + r of batch kb into buffers Q RB + r.
    template <int Q>
    __device__ __forceinline__ void load_batch(int kb) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t soff = (uint32_t)(kb * RB + r) * row_bytes;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                buf[Q * RB + r][c] = __builtin_bit_cast(
                    Raw, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(voff[c] + soff), 0, kLoadAux));
        }
    }

    // Rows (batches) 0 .. D-2 in flight (issued before anything the pass waits on).
    __device__ __forceinline__ void prime() {
        if constexpr (RB == 1) {
            if constexpr (D >= 2) load_row<0>(0);
            if constexpr (D >= 3) load_row<1>(1);
            if constexpr (D >= 4) load_row<2>(2);
        } else {
            if constexpr (D >= 2) load_batch<0>(0);
            if constexpr (D >= 3) load_batch<1>(1);
            if constexpr (D >= 4) load_batch<2>(2);
        }
    }

    __device__ __forceinline__ void load_v_regs(const double* v) {
        if constexpr (kVreg) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    int64_t j = col[c] + e;
                    vv[c * V + e] = (j < m) ? (AT)v[j] : (AT)0;
                }
        }
    }

    __device__ __forceinline__ void clear_acc() {
#pragma unroll
        for (int e = 0; e < (kAcc ? E : 1); ++e) acc[e] = (AT)0;
    }

    // One row: dot with v (FUSED/ROW/MARG), cross-wave reduction, scaling,
    // accumulation of the column partials (FUSED/COL/MARG).
    template <int Q>
    __device__ __forceinline__ void process(const PassLaunch& L, int k, const AT* vl, const double* row_in,
                                            const double* row_sh, double (*red)[NW * RB], int& slot) {
        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        AT ur;
        if constexpr (kDot) {
            AT s = (AT)0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                AT x[V];
                Unpack<KT, AT>::run(buf[Q][c], x);
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
            tot *= L.k_scale;
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
                    if (L.s_trace) L.s_trace[r0 + k] = tot;
                    if (ai > 0.0 && !(tot > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
                    if (!isfinite(uval)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
                }
            }
            ur = (AT)uval;
            if constexpr (MODE == MODE_MATRIX) {
                if (tid == 0 && L.s_out) L.s_out[r0 + k] = uval * tot;
            }
        } else {
            ur = (AT)row_in[k];
        }
        if constexpr (MODE == MODE_MATRIX) {
            // The rescaled row x_ij beta_j alpha_i is written back in place and
            // accumulated (its column sums give the next column factors).
            static_assert(sizeof(KT) == sizeof(AT), "the in-place form keeps the storage type");
            const uint32_t soff = (uint32_t)k * row_bytes;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                AT x[V];
                Unpack<KT, AT>::run(buf[Q][c], x);
                Raw z;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    AT beta;
                    if constexpr (VLDS) beta = (col[c] < m) ? vl[col[c] + e] : (AT)0;
                    else beta = vv[c * V + e];
                    if (ragged && col[c] + e >= m) x[e] = (AT)0;
                    const AT y = (x[e] * beta) * ur;
                    z[e] = y;
                    acc[c * V + e] += y;
                }
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, z), rsrc, (int)(voff[c] + soff), 0,
                                                       0);
            }
        } else if constexpr (kAcc) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                AT x[V];
                Unpack<KT, AT>::run(buf[Q][c], x);
#pragma unroll
                for (int e = 0; e < V; ++e) acc[c * V + e] = fma(x[e], ur, acc[c * V + e]);
            }
        }
    }

    // One batch of RB rows (RB > 1): the rows' dots, one exchange, the
    // factors side by side, the accumulation.  Rows past the strip (the last
    // batch may be partial) read 0 and write nothing.
    template <int Q>
    __device__ __forceinline__ void process_batch(const PassLaunch& L, int kb, const AT* vl, const double* row_in,
                                                  const double* row_sh, double (*red)[NW * RB], int& slot) {
        static_assert(MODE != MODE_MATRIX, "the in-place form runs the one-row shapes");
        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int kl = kb * RB + (lane < RB ? lane : 0);      // lane r's row
        double ul = 0.0;
        if constexpr (kDot) {
            double d[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                AT s = (AT)0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    AT x[V];
                    Unpack<KT, AT>::run(buf[Q * RB + r][c], x);
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
                d[r] = wave_sum_f64((double)s);
            }
            if (lane == 0)
#pragma unroll
                for (int r = 0; r < RB; ++r) red[slot][r * NW + wave] = d[r];
            __syncthreads();
            // Lane r NW + w takes wave w's sum of row r; each group of NW lanes
            // adds its row's sums in a fixed tree, and lane r keeps row r's total.
            static_assert(RB * NW <= 64, "one exchange entry per lane");
            const double t = group_sum_f64<NW>(lane < RB * NW ? red[slot][lane] : 0.0);
            double tl = 0.0;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double x = readlane_f64(t, r * NW);
                if (lane == r) tl = x;
            }
            tl *= L.k_scale;
            slot ^= 1;
            if (lane < RB && kl < nrows) {
                if constexpr (MODE == MODE_MARG) {
                    ul = row_in[kl];
                    if (wave == 0) L.s_out[r0 + kl] = tl;
                } else {
                    const double ai = row_in[kl];
                    ul = scale_factor(ai, tl, L.fi, L.fi_is_one, row_sh[kl]);
                    if (wave == 0) {
                        L.u[r0 + kl] = ul;
                        if (L.s_trace) L.s_trace[r0 + kl] = tl;
                        if (ai > 0.0 && !(tl > 0.0)) atomicOr(&L.ctrl->flags, UOT_FLAG_ZERO_SUM);
                        if (!isfinite(ul)) atomicOr(&L.ctrl->flags, UOT_FLAG_NONFINITE);
                    }
                }
            }
        } else {
            if (lane < RB && kl < nrows) ul = row_in[kl];
        }
        if constexpr (kAcc) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const AT ur = (AT)readlane_f64(ul, r);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    AT x[V];
                    Unpack<KT, AT>::run(buf[Q * RB + r][c], x);
#pragma unroll
                    for (int e = 0; e < V; ++e) acc[c * V + e] = fma(x[e], ur, acc[c * V + e]);
                }
            }
        }
    }

    template <int Q>
    __device__ __forceinline__ bool step(const PassLaunch& L, int k0, const AT* vl, const double* row_in,
                                         const double* row_sh, double (*red)[NW * RB], int& slot) {
        const int k = k0 + Q;
        if constexpr (RB == 1) {
            if (k >= nrows) return false;
            load_row<(Q + D - 1) % D>(k + D - 1);
            process<Q>(L, k, vl, row_in, row_sh, red, slot);
        } else {
            if (k * RB >= nrows) return false;
            load_batch<(Q + D - 1) % D>(k + D - 1);
            process_batch<Q>(L, k, vl, row_in, row_sh, red, slot);
        }
        return true;
    }

    // All rows (batches) of the strip; expects prime() to have been called.
    __device__ __forceinline__ void stream(const PassLaunch& L, const AT* vl, const double* row_in,
                                           const double* row_sh, double (*red)[NW * RB]) {
        int slot = 0;
        const int steps = (nrows + RB - 1) / RB;
        for (int k0 = 0; k0 < steps; k0 += D) {
            if (!step<0>(L, k0, vl, row_in, row_sh, red, slot)) break;
            if constexpr (D >= 2) if (!step<1 % D>(L, k0, vl, row_in, row_sh, red, slot)) break;
            if constexpr (D >= 3) if (!step<2 % D>(L, k0, vl, row_in, row_sh, red, slot)) break;
            if constexpr (D >= 4) if (!step<3 % D>(L, k0, vl, row_in, row_sh, red, slot)) break;
        }
    }

    __device__ __forceinline__ void store_partials(AT* P) {
        if constexpr (kAcc) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (col[c] >= m) continue;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    // ldp is a multiple of 64 >= m, so the chunk lies inside the partial
                    // row; streaming stores: the partials are read once, elsewhere.
                    __builtin_nontemporal_store(acc[c * V + e], &P[col[c] + e]);
                }
            }
        }
    }
};

// Stage the strip's per-row inputs (a and the stabilised shift, or u) and,
// for shapes that keep v in LDS, v itself.
template <typename S, int MODE, bool VLDS, typename AT>
__device__ __forceinline__ void stage_rows(const PassLaunch& L, int64_t r0, int nrows, double* row_in,
                                           double* row_sh) {
    for (int k = threadIdx.x; k < nrows; k += blockDim.x) {
        if constexpr (MODE == MODE_FUSED || MODE == MODE_ROW || MODE == MODE_MATRIX) {
            row_in[k] = L.a[r0 + k];
            row_sh[k] = L.fpot ? -(1.0 - L.fi) * L.fpot[r0 + k] * L.inv_eps : 0.0;
        } else {
            row_in[k] = L.u[r0 + k];
        }
    }
}

// v (FP64) into LDS as AT.  Each lane issues its kStageV loads before the
// first wait (a loop that waited on each load in turn would put that many L2
// round trips in front of the workgroup's first row).  The loads go through a
// buffer resource over v (entries j >= m read as 0; the whole offset is the
// lane's, so the range check covers it).  Requires 8 m < 2^31 (v fits in LDS
// here).
constexpr int kStageV = 16;

template <int V, int NT, typename AT>
__device__ __forceinline__ void stage_v(const double* v, int64_t m, AT* vl) {
    const int mv = (int)((m + V - 1) / V * V);
    constexpr int nt = NT;
    const __amdgpu_buffer_rsrc_t vr = __builtin_amdgcn_make_buffer_rsrc((void*)v, (short)0, (int)(m * 8), kBufferWord3);
    for (int j0 = threadIdx.x; j0 < mv; j0 += nt * kStageV) {
        double x[kStageV];
#pragma unroll
        for (int q = 0; q < kStageV; ++q)
            x[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(vr, (j0 + q * nt) * 8, 0, 0));
#pragma unroll
        for (int q = 0; q < kStageV; ++q) {
            const int j = j0 + q * nt;
            if (j < mv) vl[j] = (AT)x[q];
        }
    }
}

// Stopping test of the previous iteration (see PassLaunch): identical in
// every workgroup.  Returns true when the loop is to stop.
// Early exit of a per-iteration pass launch, the same for every wave of the
// workgroup.  The stop flag can change during a launch only when that launch
// applies the stopping test (block 0 then sets it), so in that case wave 0
// alone reads the flag and evaluates the test, and one barrier hands the
// decision to the other waves; otherwise the flag is fixed for the whole
// launch and every wave reads it directly.
__device__ __forceinline__ bool pass_exit(const PassLaunch& L, uint32_t* exit_sh) {
    const bool test = L.test_stop && L.tol > 0.0 && L.iter > 1;
    if (!test) return L.check_done && ld_volatile_u32(&L.ctrl->done) != 0;
    if (threadIdx.x < 64) {
        const uint32_t flag = L.check_done ? ld_volatile_u32(&L.ctrl->done) : 0u;
        bool quit = __builtin_amdgcn_readfirstlane(flag) != 0;
        if (!quit) {
            const double err = stop_error(L.blockpart, L.fin_blocks, threadIdx.x);
            quit = err <= L.tol;
            if (quit && blockIdx.x == 0 && threadIdx.x == 0) {
                L.ctrl->iters = L.iter - 1;
                L.ctrl->err = err;
                L.ctrl->done = 1;
            }
        }
        if (threadIdx.x == 0) *exit_sh = quit ? 1u : 0u;
    }
    __syncthreads();
    return *exit_sh != 0;
}

// Stopping test of the cooperative loop: every wave of every workgroup
// evaluates it at the same point (no early flag read).
__device__ __forceinline__ bool stop_test(const PassLaunch& L, int64_t iter, double* err_sh) {
    if (!(L.tol > 0.0) || iter <= 1) return false;
    if ((threadIdx.x >> 6) == 0) {
        double err = stop_error(L.blockpart, L.fin_blocks, threadIdx.x & 63);
        if ((threadIdx.x & 63) == 0) *err_sh = err;
    }
    __syncthreads();
    const double err = *err_sh;
    __syncthreads();
    if (err <= L.tol) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            L.ctrl->iters = iter - 1;
            L.ctrl->err = err;
            L.ctrl->done = 1;
        }
        return true;
    }
    return false;
}

}  // namespace uot
