// Reverse mode through the unrolled UOT Sinkhorn iteration.
//
// The forward iteration (paper Section 2.1 on scaling vectors; rows first
// from v_0 = 1) is t = 1..T:  s_t = K v_{t-1}, u_t = (a/s_t)^fi,
// w_t = K^T u_t, v_t = (b/w_t)^fi, and the objective is
//   L = eps (sum r log u_T + sum c log v_T - sum r) + tau KL~(r|a) + tau KL~(c|b),
// r = u_T * (K v_T), c = v_T * (K^T u_T).  Its exact gradient:
//
// seeds   rbar = eps log u + tau log(r/a) - eps,   cbar = eps log v + tau log(c/b)
//         ubar_T = eps K v + rbar * K v + K (cbar * v)
//         vbar_T = eps K^T u + K^T (rbar * u) + cbar * K^T u
//         Kbar  = (rbar * u) v^T + u (cbar * v)^T,   abar = tau (1 - r/a),  bbar = tau (1 - c/b)
// step t  wbar = -fi vbar_t * v_t / w_t;   bbar += fi vbar_t * v_t / b
//         ubar_t = K wbar (+ ubar_T at t = T);   Kbar += u_t wbar^T
//         sbar = -fi ubar_t * u_t / s_t;   abar += fi ubar_t * u_t / a
//         vbar_{t-1} = K^T sbar;   Kbar += sbar v_{t-1}^T
//
// dL/dC = -Kbar * K / eps is never formed: for a squared-Euclidean cost of
// points, dL/dx_i = 2 (x_i sum_j G_ij - sum_j G_ij y_j), G = dL/dC, and both
// row sums follow from extra right-hand sides of the same row pass:
//   sum_j K_ij Kbar_ij (1, y_j) = u_i (K (wbar*(1,y)))_i + sbar_i (K (v_{t-1}*(1,y)))_i.
//
// One adjoint pass per step streams K once (row dots with A = wbar and
// B = v_{t-1}, times 1 and each coordinate of y; then the column partials of
// K^T sbar), so a reverse step costs what a forward iteration costs.
#include "strip.h"

namespace uot {

// Totals over a 512-lane workgroup of ND <= 8 per-lane values, FP64, in a
// fixed order; every lane returns the same T.
//  1. Within each 16-lane row, a transposing butterfly: at each level a lane
//     keeps half of its values and sends the other half to its partner (row
//     mirror, half-row mirror, lane ^ 2), so ND values cost 4 + 2 + 1 moves
//     instead of 4 per value; after a last lane ^ 1 exchange, lanes 2p and
//     2p + 1 of a row hold the row's sum of value p = (lane >> 1) & 7.
//  2. Even lanes write their sum to red[p][4 wave + row]; one barrier.
//  3. Lane l adds the 4 entries red[l >> 3][4 (l & 7) .. +3] in order, then
//     the 8 lanes of each group finish with three exchanges (lane ^ 1,
//     lane ^ 2, half-row mirror) and T[p] is read from lane 8 p.
template <int ND>
__device__ __forceinline__ void block_sums8(const double (&x)[ND], double (*red)[32], int lane, int wave,
                                            double (&T)[ND]) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = q < ND ? x[q] : 0.0;
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0;
    double a[4], b[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double keep = b3 ? v[j + 4] : v[j];
        const double send = b3 ? v[j] : v[j + 4];
        a[j] = keep + dpp_f64<0x140>(send);       // row_mirror: lane i <-> 15 - i
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double keep = b2 ? a[j + 2] : a[j];
        const double send = b2 ? a[j] : a[j + 2];
        b[j] = keep + dpp_f64<0x141>(send);       // row_half_mirror: i <-> 7 - i in each half
    }
    double c;
    {
        const double keep = b1 ? b[1] : b[0];
        const double send = b1 ? b[0] : b[1];
        c = keep + dpp_f64<0x4E>(send);           // lane ^ 2
    }
    c += dpp_f64<0xB1>(c);                         // lane ^ 1
    if (!(lane & 1)) red[(lane >> 1) & 7][4 * wave + (lane >> 4)] = c;
    __syncthreads();
    const double* p = &red[lane >> 3][4 * (lane & 7)];
    double t = ((p[0] + p[1]) + p[2]) + p[3];
    t += dpp_f64<0xB1>(t);
    t += dpp_f64<0x4E>(t);
    t += dpp_f64<0x141>(t);
#pragma unroll
    for (int q = 0; q < ND; ++q) T[q] = readlane_f64(t, 8 * q);
}

template <typename KT, typename AT, int WG, int NC, int D, int DIM, int PHASE>
__global__ __launch_bounds__(WG) void adj_kernel(AdjLaunch L) {
    using S = Strip<KT, AT, WG, NC, D, false, MODE_COL>;
    using Raw = typename S::Raw;
    constexpr int V = S::V;
    constexpr int E = S::E;
    constexpr int NW = WG / 64;
    constexpr bool kB = (PHASE == ADJ_SEED) || (DIM > 0);   // dots with B needed
    constexpr int ND = 2 + 2 * DIM;                         // dA, dB, dAy[DIM], dBy[DIM]
    static_assert(NW == 8 && ND <= 8, "the row reduction maps 8 values x 8 waves onto 64 lanes");
    __shared__ double red[2][8][32];
    extern __shared__ __align__(16) unsigned char dyn_lds[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * L.rows_per_wg;
    int64_t r1 = r0 + L.rows_per_wg;
    if (r1 > L.n) r1 = L.n;
    const int nrows = (int)(r1 - r0);
    const int64_t m = L.m;

    PassLaunch P;
    P.K = L.K;
    P.ldk = L.ldk;
    P.m = L.m;
    S st;
    st.setup(P, r0, nrows);
    st.prime();

    // LDS per row of the strip: u, s, a, useed, abar, gsum, gy[DIM]
    const int R = (int)L.rows_per_wg;
    double* lu = (double*)dyn_lds;
    double* ls = lu + R;
    double* la = ls + R;
    double* lseed = la + R;
    double* labar = lseed + R;
    double* lgsum = labar + R;
    double* lgy = lgsum + R;
    for (int k = tid; k < nrows; k += WG) {
        const int64_t i = r0 + k;
        lu[k] = L.u[i];
        la[k] = L.a[i];
        if constexpr (PHASE == ADJ_STEP) {
            ls[k] = L.s[i];
            lseed[k] = L.add_seed ? L.useed[i] : 0.0;
            labar[k] = L.abar[i];
            if constexpr (DIM > 0) {
                lgsum[k] = L.gsum[i];
#pragma unroll
                for (int d = 0; d < DIM; ++d) lgy[k * DIM + d] = L.gy[i * DIM + d];
            }
        }
    }

    // Coordinates of y in LDS, one contiguous row per coordinate (after the
    // per-row arrays): yl[d * mp + j].
    // yl starts on a 16-byte boundary so that V consecutive entries load as one vector.
    const int64_t mp = (m + V - 1) / V * V;
    const size_t yl_off = (sizeof(double) * (size_t)R * (6 + (DIM > 0 ? DIM : 1)) + 15) & ~(size_t)15;
    AT* yl = (AT*)(dyn_lds + yl_off);
    if constexpr (DIM > 0) {
        // Loads of U points issued before the first wait (indices clamped in bounds).
        constexpr int U = 4;
        for (int64_t j0 = tid; j0 < mp; j0 += (int64_t)WG * U) {
            double x[U][DIM];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int64_t j = j0 + (int64_t)q * WG;
                const int64_t jc = j < m ? j : m - 1;
#pragma unroll
                for (int d = 0; d < DIM; ++d) x[q][d] = L.y[jc * DIM + d];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int64_t j = j0 + (int64_t)q * WG;
                if (j < mp)
#pragma unroll
                    for (int d = 0; d < DIM; ++d) yl[d * mp + j] = (j < m) ? (AT)x[q][d] : (AT)0;
            }
        }
    }
    // Right-hand sides of this lane's columns.
    AT Av[E], Bv[kB ? E : 1];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int64_t j = st.col[c] + e;
            const bool in = j < m;
            Av[c * V + e] = in ? (AT)L.A[j] : (AT)0;
            if constexpr (kB) Bv[c * V + e] = in ? (AT)L.B[j] : (AT)0;
        }
    st.clear_acc();
    __syncthreads();

    const double inv_eps = 1.0 / L.eps;
    int slot = 0;
    auto process = [&](Raw (&b)[NC], int k) {
        AT dA = 0, dB = 0, dAy[DIM > 0 ? DIM : 1], dBy[DIM > 0 ? DIM : 1];
#pragma unroll
        for (int d = 0; d < (DIM > 0 ? DIM : 1); ++d) dAy[d] = dBy[d] = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            AT x[V];
            Unpack<KT, AT>::run(b[c], x);
            if (st.ragged) {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (st.col[c] + e >= m) x[e] = (AT)0;
            }
            // The chunk's coordinates as one 16-byte LDS read per dimension.  A
            // chunk past column m reads the last chunk instead (in bounds); its
            // K entries and right-hand sides are 0, so it adds nothing.
            AT yv[DIM > 0 ? DIM : 1][V];
            if constexpr (DIM > 0) {
                const int jc = (int)(st.col[c] < mp ? st.col[c] : mp - V);
#pragma unroll
                for (int d = 0; d < DIM; ++d)
                    Unpack<AT, AT>::run(*(const Raw*)&yl[d * mp + jc], yv[d]);
            }
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int q = c * V + e;
                const AT tA = x[e] * Av[q];
                dA += tA;
                AT tB = (AT)0;
                if constexpr (kB) {
                    tB = x[e] * Bv[q];
                    dB += tB;
                }
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    dAy[d] = fma(tA, yv[d][e], dAy[d]);
                    dBy[d] = fma(tB, yv[d][e], dBy[d]);
                }
            }
        }
        double part[ND];
        part[0] = (double)dA;
        part[1] = (double)dB;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            part[2 + d] = (double)dAy[d];
            part[2 + DIM + d] = (double)dBy[d];
        }
        double T[ND];
        block_sums8<ND>(part, red[slot], lane, wave, T);
        slot ^= 1;
        const double ui = lu[k], ai = la[k];
        double qrow;
        if constexpr (PHASE == ADJ_SEED) {
            // T[0] = (K (cbar v))_i, T[1] = (K v_T)_i
            double rbar = 0.0, useed = 0.0, abar = 0.0;
            if (ui > 0.0) {
                const double r = ui * T[1];
                rbar = L.eps * log(ui) - L.eps + (L.tau_inf ? 0.0 : L.tau * log(r / ai));
                useed = L.eps * T[1] + rbar * T[1] + T[0];
                abar = L.tau_inf ? 0.0 : L.tau * (1.0 - r / ai);
            }
            qrow = rbar * ui;
            if (tid == 0) {
                if (L.st_q) L.st_q[r0 + k] = qrow;
                lseed[k] = useed;
                labar[k] = abar;
                if constexpr (DIM > 0) {
                    lgsum[k] = -inv_eps * (rbar * ui * T[1] + ui * T[0]);
#pragma unroll
                    for (int d = 0; d < DIM; ++d)
                        lgy[k * DIM + d] = -inv_eps * (rbar * ui * T[2 + DIM + d] + ui * T[2 + d]);
                }
            }
        } else {
            // T[0] = (K wbar)_i, T[1] = (K v_{t-1})_i = s_t,i
            const double ubar = T[0] + lseed[k];
            const double si = ls[k];
            const double sbar = (ui > 0.0) ? -L.fi * ubar * ui / si : 0.0;
            qrow = sbar;
            if (tid == 0) {
                if (L.st_q) L.st_q[r0 + k] = qrow;
                if (ai > 0.0) labar[k] += L.fi * ubar * ui / ai;
                if constexpr (DIM > 0) {
                    lgsum[k] += -inv_eps * (ui * T[0] + sbar * T[1]);
#pragma unroll
                    for (int d = 0; d < DIM; ++d) lgy[k * DIM + d] += -inv_eps * (ui * T[2 + d] + sbar * T[2 + DIM + d]);
                }
            }
        }
        const AT qa = (AT)qrow;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            AT x[V];
            Unpack<KT, AT>::run(b[c], x);
#pragma unroll
            for (int e = 0; e < V; ++e) st.acc[c * V + e] = fma(x[e], qa, st.acc[c * V + e]);
        }
    };

    static_assert(D == 2, "the adjoint pass is pipelined two rows deep");
    for (int k0 = 0; k0 < nrows; k0 += 2) {
        st.template load_row<1>(k0 + 1);
        process(st.buf[0], k0);
        if (k0 + 1 >= nrows) break;
        st.template load_row<0>(k0 + 2);
        process(st.buf[1], k0 + 1);
    }

    __syncthreads();
    for (int k = tid; k < nrows; k += WG) {
        const int64_t i = r0 + k;
        if (L.st_u) L.st_u[i] = lu[k];
        if constexpr (PHASE == ADJ_SEED) L.useed[i] = lseed[k];
        L.abar[i] = labar[k];
        if constexpr (DIM > 0) {
            L.gsum[i] = lgsum[k];
#pragma unroll
            for (int d = 0; d < DIM; ++d) L.gy[i * DIM + d] = lgy[k * DIM + d];
        }
    }
    st.store_partials((AT*)L.partials + (int64_t)blockIdx.x * L.ldp);
    if (L.st_a) {
        // Column factors: each workgroup copies its share of A and B.
        const int64_t per = (m + gridDim.x - 1) / gridDim.x;
        const int64_t j0 = (int64_t)blockIdx.x * per;
        const int64_t j1 = j0 + per < m ? j0 + per : m;
        for (int64_t j = j0 + tid; j < j1; j += WG) {
            L.st_a[j] = L.A[j];
            L.st_b[j] = L.B[j];
        }
    }
}

size_t adj_lds_bytes(int64_t rows_per_wg, int dim, int64_t m, int elem) {
    const int64_t mp = (m + 15) / 16 * 16;
    return sizeof(double) * (size_t)rows_per_wg * (6 + (size_t)(dim > 0 ? dim : 1)) + (size_t)elem * mp * dim + 16;
}

template <typename KT, typename AT, int WG, int NC, int DIM>
static hipError_t adj_launch_dim(int phase, const AdjLaunch& L, hipStream_t stream) {
    const size_t lds = adj_lds_bytes(L.rows_per_wg, DIM, L.m, (int)sizeof(AT));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)adj_kernel<KT, AT, WG, NC, 2, DIM, ADJ_SEED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)adj_kernel<KT, AT, WG, NC, 2, DIM, ADJ_STEP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (phase == ADJ_SEED)
        hipLaunchKernelGGL((adj_kernel<KT, AT, WG, NC, 2, DIM, ADJ_SEED>), dim3(L.grid), dim3(WG), lds, stream, L);
    else
        hipLaunchKernelGGL((adj_kernel<KT, AT, WG, NC, 2, DIM, ADJ_STEP>), dim3(L.grid), dim3(WG), lds, stream, L);
    return hipGetLastError();
}

template <typename KT, typename AT, int WG, int NC>
static hipError_t adj_launch_nc(int phase, int dim, const AdjLaunch& L, hipStream_t stream) {
    switch (dim) {
        case 0: return adj_launch_dim<KT, AT, WG, NC, 0>(phase, L, stream);
        case 2: return adj_launch_dim<KT, AT, WG, NC, 2>(phase, L, stream);
        case 3: return adj_launch_dim<KT, AT, WG, NC, 3>(phase, L, stream);
        default: return hipErrorInvalidValue;
    }
}

// 512-lane workgroups (two waves per SIMD, 256 VGPRs): each lane holds A, B
// and the coordinates of y for its columns in registers.
int adj_chunks_max(int k_dtype) { return 4; }
int adj_wg() { return 512; }

hipError_t launch_adj(int k_dtype, int nc, int phase, int dim, const AdjLaunch& L, hipStream_t stream) {
    if (k_dtype == UOT_F32) {
        if (nc == 1) return adj_launch_nc<float, float, 512, 1>(phase, dim, L, stream);
        if (nc == 2) return adj_launch_nc<float, float, 512, 2>(phase, dim, L, stream);
        if (nc == 4) return adj_launch_nc<float, float, 512, 4>(phase, dim, L, stream);
    } else if (k_dtype == UOT_F64) {
        if (nc == 1) return adj_launch_nc<double, double, 512, 1>(phase, dim, L, stream);
        if (nc == 2) return adj_launch_nc<double, double, 512, 2>(phase, dim, L, stream);
        if (nc == 4) return adj_launch_nc<double, double, 512, 4>(phase, dim, L, stream);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Column side of the reverse pass: sums of the partials (fixed order, FP64)
// and the O(m) updates around them.
//   ADJ_COL_PREP  w = K^T u_T; c = v w; cbar, h = cbar * v (the seed pass's A), bbar = tau(1 - c/b)
//   ADJ_COL_SEED  vbar_T = sum + eps w + cbar w; then the step-T update below
//   ADJ_COL_STEP  vbar_{t-1} = sum; then wbar = -fi vbar v / w, bbar += fi vbar v / b
// ---------------------------------------------------------------------------
constexpr int ACOL_COLS = 16;
constexpr int ACOL_THREADS = 256;
constexpr int ACOL_PHASES = ACOL_THREADS / (ACOL_COLS / 4);

template <typename AT>
__global__ __launch_bounds__(ACOL_THREADS) void adj_col_kernel(AdjColLaunch C) {
    __shared__ double part[ACOL_PHASES][ACOL_COLS + 1];
    const int tid = threadIdx.x;
    const int cg = tid & (ACOL_COLS / 4 - 1);
    const int ph = tid / (ACOL_COLS / 4);
    const int64_t c0 = (int64_t)blockIdx.x * ACOL_COLS + 4 * cg;
    const AT* Pp = (const AT*)C.partials + c0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (c0 < C.m) {
        for (int g = ph; g < C.G; g += ACOL_PHASES) {
            double x[4];
            Chunk4<AT>::load(Pp + (int64_t)g * C.ldp, x);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += x[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[ph][4 * cg + e] = acc[e];
    __syncthreads();
    if (tid >= ACOL_COLS) return;
    const int64_t j = (int64_t)blockIdx.x * ACOL_COLS + tid;
    if (j >= C.m) return;
    double sum = 0.0;
    for (int k = 0; k < ACOL_PHASES; ++k) sum += part[k][tid];
    const double vj = C.v[j], bj = C.b[j];
    if (C.mode == ADJ_COL_PREP) {
        const double w = sum;
        const double c = vj * w;
        double cbar = 0.0, bbar = 0.0;
        if (vj > 0.0) {
            cbar = C.eps * log(vj) + (C.tau_inf ? 0.0 : C.tau * log(c / bj));
            bbar = C.tau_inf ? 0.0 : C.tau * (1.0 - c / bj);
        }
        C.w[j] = w;
        C.cbar[j] = cbar;
        C.out[j] = cbar * vj;
        C.bbar[j] = bbar;
        return;
    }
    double vbar = sum;
    if (C.mode == ADJ_COL_SEED) vbar += C.eps * C.w[j] + C.cbar[j] * C.w[j];
    double wbar = 0.0;
    if (vj > 0.0) {
        wbar = -C.fi * vbar * vj / C.w[j];
        C.bbar[j] += C.fi * vbar * vj / bj;
    }
    C.out[j] = wbar;
}

hipError_t launch_adj_col(const AdjColLaunch& C, hipStream_t stream) {
    dim3 grid((unsigned)((C.m + ACOL_COLS - 1) / ACOL_COLS)), block(ACOL_THREADS);
    if (C.acc64)
        hipLaunchKernelGGL(adj_col_kernel<double>, grid, block, 0, stream, C);
    else
        hipLaunchKernelGGL(adj_col_kernel<float>, grid, block, 0, stream, C);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final scaling by dLoss: grad_a = g abar, grad_b = g bbar,
// grad_x_i = 2 g (x_i gsum_i - gy_i).
// ---------------------------------------------------------------------------
__global__ void adj_finish_kernel(AdjFinish F) {
    const double g = *F.grad_loss;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = t; i < F.n; i += stride) {
        if (F.grad_a) F.grad_a[i] = g * F.abar[i];
        if (F.grad_x)
            for (int d = 0; d < F.dim; ++d)
                F.grad_x[i * F.dim + d] = 2.0 * g * (F.x[i * F.dim + d] * F.gsum[i] - F.gy[i * F.dim + d]);
    }
    for (int64_t j = t; j < F.m; j += stride)
        if (F.grad_b) F.grad_b[j] = g * F.bbar[j];
}

hipError_t launch_adj_finish(const AdjFinish& F, hipStream_t stream) {
    int64_t mx = F.n > F.m ? F.n : F.m;
    int blocks = (int)((mx + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(adj_finish_kernel, dim3(blocks), dim3(256), 0, stream, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cost gradient.  Kbar is the sum of 2T + 2 rank-1 terms whose factors the
// reverse passes stored (slot s: row factor Lf[s], column factor Rf[s]), so
//   dL/dC_ij = -(grad_loss / eps) K_ij sum_s Lf[s][i] Rf[s][j]
// is one dense FP64 product with inner dimension 2T + 2 (a contraction: it
// runs on the matrix cores, v_mfma_f64_16x16x4f64) and the kernel applied in
// its epilogue.  Workgroup: 4 waves in 2 x 2 over a 128 x 128 output tile,
// each wave 64 x 64 as 4 x 4 blocks of 16 x 16.  The factors of 16 slots
// (16 KiB of Lf and of Rf, each slot's 128 entries one contiguous 1 KiB run)
// are staged through LDS, double buffered: the next slab's loads are in
// flight while the 64 products of the current one issue, and one barrier
// separates slabs.  Fragment of a block (16 rows x 4 slots): lane l holds
// Lf[s0 + l/16][i0 + l%16].  Slots are padded to a multiple of 16 and rows to
// multiples of 128 with zero factors (kGradcSlotPad, kGradcRowPad).  Output block: lane l
// holds rows i0 + l/16 + 4 q, q < 4, of column j0 + l%16 (the FP64 form
// interleaves its four result rows, unlike the FP32 16 x 16 forms).
// ---------------------------------------------------------------------------
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int GC_WG = 256;
constexpr int GC_TILE = kGradcRowPad;
constexpr int GC_KS = kGradcSlotPad;    // slots per LDS slab

int gradc_row_tiles(int64_t n) { return (int)((n + GC_TILE - 1) / GC_TILE); }

__global__ void fill_f64_kernel(double* p, int64_t count, double value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) p[k] = value;
}

hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, count, value);
    return hipGetLastError();
}

template <typename KT, int DIM>
__global__ __launch_bounds__(GC_WG, 2) void gradc_kernel(GradCLaunch L) {
    constexpr int ND = 1 + DIM;
    __shared__ double red[2][ND][64];
    __shared__ __align__(16) double As[2][GC_KS][GC_TILE];
    __shared__ __align__(16) double Bs[2][GC_KS][GC_TILE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t n = L.n, m = L.m;
    const int64_t ldl = L.ldl, ldr = L.ldr;     // padded row lengths of Lf, Rf
    const int64_t tiles_j = (m + GC_TILE - 1) / GC_TILE;
    const int64_t tiles = tiles_j * ((n + GC_TILE - 1) / GC_TILE);
    // Workgroups go to the 8 XCDs in turn: give each XCD a contiguous run of
    // tiles (same row tile, so its row factors stay in that XCD's L2).
    int64_t b = blockIdx.x;
    if (tiles % 8 == 0) b = (b % 8) * (tiles / 8) + b / 8;
    const int64_t ti = b / tiles_j, tj = b % tiles_j;
    const int64_t it0 = ti * GC_TILE, jt0 = tj * GC_TILE;
    const int64_t i0 = it0 + wi * 64;
    const int64_t j0 = jt0 + wj * 64;
    const int r16 = lane & 15, g4 = lane >> 4;

    // Slab loads: thread t moves 8 consecutive factors (four 16-byte loads)
    // of slot t/16 for Lf and for Rf.
    const int ls = tid >> 4, lc = (tid & 15) * 8;
    const double* ga = L.Lf + (int64_t)ls * ldl + it0 + lc;
    const double* gb = L.Rf + (int64_t)ls * ldr + jt0 + lc;
    f64x2 ra[4], rb[4];
    auto fetch = [&](int64_t slab) {
        const double* pa = ga + slab * GC_KS * ldl;
        const double* pb = gb + slab * GC_KS * ldr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ra[q] = *(const f64x2*)(pa + 2 * q);
            rb[q] = *(const f64x2*)(pb + 2 * q);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *(f64x2*)&As[buf][ls][lc + 2 * q] = ra[q];
            *(f64x2*)&Bs[buf][ls][lc + 2 * q] = rb[q];
        }
    };

    f64x4_t acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = (f64x4_t){0.0, 0.0, 0.0, 0.0};

    const int64_t slabs = L.nterms / GC_KS;     // nterms is padded to a multiple of GC_KS
    fetch(0);
    stash(0);
    __syncthreads();
    for (int64_t sl = 0; sl < slabs; ++sl) {
        const int buf = (int)(sl & 1);
        if (sl + 1 < slabs) fetch(sl + 1);
#pragma unroll
        for (int kk = 0; kk < GC_KS / 4; ++kk) {
            double a[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[buf][4 * kk + g4][wi * 64 + 16 * q + r16];
                bv[q] = Bs[buf][4 * kk + g4][wj * 64 + 16 * q + r16];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], bv[q], acc[p][q], 0, 0, 0);
        }
        if (sl + 1 < slabs) stash(buf ^ 1);
        __syncthreads();
    }

    // Epilogue: G = scale K (.) acc; column sums of G and G x_i for the target gradient.
    const double scale = -(*L.grad_loss) * L.inv_eps;
    const KT* Kp = (const KT*)L.K;
    double cs[4][ND];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int d = 0; d < ND; ++d) cs[q][d] = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + 16 * p + g4 + 4 * e;
            if (i >= n) continue;
            double xi[DIM > 0 ? DIM : 1];
            if constexpr (DIM > 0) {
                if (L.ysum)
#pragma unroll
                    for (int d = 0; d < DIM; ++d) xi[d] = L.x[i * DIM + d];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t j = j0 + 16 * q + r16;
                if (j >= m) continue;
                const double g = scale * (double)Kp[i * L.ldk + j] * acc[p][q][e];
                if (L.G) L.G[i * L.ldg + j] = g;
                cs[q][0] += g;
#pragma unroll
                for (int d = 0; d < DIM; ++d) cs[q][1 + d] += g * xi[d];
            }
        }
    }
    if (!L.ysum) return;
    // Sum the 4 row groups of the wave, then the two waves of a column range.
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double v = cs[q][d];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            cs[q][d] = v;
        }
    if (wi == 1 && g4 == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int d = 0; d < ND; ++d) red[wj][d][16 * q + r16] = cs[q][d];
    __syncthreads();
    if (wi == 0 && g4 == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t j = j0 + 16 * q + r16;
            if (j >= m) continue;
#pragma unroll
            for (int d = 0; d < ND; ++d) L.ysum[(ti * ND + d) * m + j] = cs[q][d] + red[wj][d][16 * q + r16];
        }
    }
}

template <typename KT>
static hipError_t gradc_launch_t(const GradCLaunch& L, hipStream_t stream) {
    const int64_t tiles = (int64_t)gradc_row_tiles(L.n) * ((L.m + GC_TILE - 1) / GC_TILE);
    const int dim = L.ysum ? L.dim : 0;
    switch (dim) {
        case 0: hipLaunchKernelGGL((gradc_kernel<KT, 0>), dim3((unsigned)tiles), dim3(GC_WG), 0, stream, L); break;
        case 2: hipLaunchKernelGGL((gradc_kernel<KT, 2>), dim3((unsigned)tiles), dim3(GC_WG), 0, stream, L); break;
        case 3: hipLaunchKernelGGL((gradc_kernel<KT, 3>), dim3((unsigned)tiles), dim3(GC_WG), 0, stream, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gradc(const GradCLaunch& L, hipStream_t stream) {
    if (L.nterms % GC_KS != 0 || L.nterms < GC_KS || L.ldl % GC_TILE != 0 || L.ldr % GC_TILE != 0 ||
        L.ldl < L.n || L.ldr < L.m)
        return hipErrorInvalidValue;
    if (L.k_dtype == UOT_F32) return gradc_launch_t<float>(L, stream);
    if (L.k_dtype == UOT_F64) return gradc_launch_t<double>(L, stream);
    return hipErrorInvalidValue;
}

__global__ void grady_finish_kernel(const double* ysum, int32_t tiles, const double* y, int64_t m, int32_t dim,
                                    double* grad_y) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int nd = 1 + dim;
    double s0 = 0.0;
    for (int t = 0; t < tiles; ++t) s0 += ysum[((int64_t)t * nd) * m + j];
    for (int d = 0; d < dim; ++d) {
        double sd = 0.0;
        for (int t = 0; t < tiles; ++t) sd += ysum[((int64_t)t * nd + 1 + d) * m + j];
        grad_y[j * dim + d] = 2.0 * (y[j * dim + d] * s0 - sd);
    }
}

hipError_t launch_grady_finish(const double* ysum, int32_t tiles, const double* y, int64_t m, int32_t dim,
                               double* grad_y, hipStream_t stream) {
    hipLaunchKernelGGL(grady_finish_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, ysum, tiles, y,
                       m, dim, grad_y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Implicit (envelope) gradients from the marginal passes:
//   s = K v, w = K^T u (one marginal pass),  sy_d = K (v y_d), wx_d = K^T (u x_d)
//   (one marginal pass per point coordinate d), then
//   grad_a = g tau (1 - u s / a), grad_b = g tau (1 - v w / b),
//   grad_x_id = 2 g (x_id u_i s_i - u_i sy_d,i),  grad_y_jd = 2 g (y_jd v_j w_j - v_j wx_d,j).
// ---------------------------------------------------------------------------
__global__ void env_weight_kernel(const double* u, const double* x, int64_t n, const double* v, const double* y,
                                  int64_t m, int32_t dim, int32_t d, double* ud, double* vd) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < n; i += stride) ud[i] = u[i] * x[i * dim + d];
    for (int64_t j = t; j < m; j += stride) vd[j] = v[j] * y[j * dim + d];
}

hipError_t launch_env_weight(const double* u, const double* x, int64_t n, const double* v, const double* y, int64_t m,
                             int32_t dim, int32_t d, double* ud, double* vd, hipStream_t stream) {
    const int64_t mx = n > m ? n : m;
    int blocks = (int)((mx + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(env_weight_kernel, dim3(blocks), dim3(256), 0, stream, u, x, n, v, y, m, dim, d, ud, vd);
    return hipGetLastError();
}

__global__ void env_finish_kernel(EnvFinish F) {
    const double g = *F.grad_loss;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < F.n; i += stride) {
        const double r = F.u[i] * F.s[i];
        if (F.grad_a) F.grad_a[i] = F.tau_inf ? 0.0 : g * F.tau * (1.0 - r / F.a[i]);
        if (F.grad_x)
            for (int d = 0; d < F.dim; ++d)
                F.grad_x[i * F.dim + d] = 2.0 * g * (F.x[i * F.dim + d] * r - F.u[i] * F.sy[(int64_t)d * F.n + i]);
    }
    for (int64_t j = t; j < F.m; j += stride) {
        const double c = F.v[j] * F.w[j];
        if (F.grad_b) F.grad_b[j] = F.tau_inf ? 0.0 : g * F.tau * (1.0 - c / F.b[j]);
        if (F.grad_y)
            for (int d = 0; d < F.dim; ++d)
                F.grad_y[j * F.dim + d] = 2.0 * g * (F.y[j * F.dim + d] * c - F.v[j] * F.wx[(int64_t)d * F.m + j]);
    }
}

hipError_t launch_env_finish(const EnvFinish& F, hipStream_t stream) {
    const int64_t mx = F.n > F.m ? F.n : F.m;
    int blocks = (int)((mx + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(env_finish_kernel, dim3(blocks), dim3(256), 0, stream, F);
    return hipGetLastError();
}

}  // namespace uot
