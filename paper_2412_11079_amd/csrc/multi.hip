// Many right-hand sides sharing one kernel K: the two half-steps of an
// iteration (Section 2.1's row and column rescaling, for R histogram pairs
// at once) become two matrix products,
//     S = K V,    U = (A / S)^fi          (n x R)
//     W = K^T U,  V = (B / W)^fi          (m x R)
// on the matrix cores.  K^T is stored once (a transposed copy in the
// workspace), so both products read their big operand with the reduction
// index contiguous.  Right-hand sides are held k-contiguous (one row per
// histogram).
//
// Two forms:
//   BF16: K stored in bfloat16; each right-hand side is split into a
//         bfloat16 high part and the bfloat16 rounding of the remainder, and
//         both go through v_mfma_f32_32x32x16_bf16 (products exact, FP32
//         accumulation), so the right-hand sides keep ~16 significant bits;
//   FP32: K and right-hand sides in FP32 through v_mfma_f32_32x32x2_f32.
// The reduction is split over k into chunks whose FP32 sums are added in
// FP64, in a fixed order, by the epilogue that also applies the power.
#include <math.h>

#include "multi.h"
#include "strip.h"

namespace uot {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Workgroup: 4 waves in a 2 x 2 arrangement; each wave owns 64 rows x 64
// right-hand sides = 2 x 2 tiles of 32 x 32.
template <bool BF>
__global__ __launch_bounds__(256) void mgemm_kernel(MGemm G) {
    constexpr int EA = BF ? 2 : 4;          // bytes per element
    constexpr int STEP = BF ? 16 : 8;       // k per step
    constexpr int KL = BF ? 8 : 4;          // k values a lane loads per operand per step
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int lr = l & 31;
    const int lh = l >> 5;
    const int64_t row0 = (int64_t)blockIdx.y * kMTileRows + (w & 1) * 64;
    const int64_t col0 = (int64_t)blockIdx.x * kMTileCols + (w >> 1) * 64;
    const int64_t k_begin = (int64_t)blockIdx.z * G.kchunk;
    int64_t k_end = k_begin + G.kchunk;
    if (k_end > G.kdim_pad) k_end = G.kdim_pad;

    const uint32_t a_bytes = (uint32_t)(G.rows * G.lda * EA);
    const uint32_t x_bytes = (uint32_t)(G.r_pad * G.ldx * EA);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void*)G.A, (short)0, (int)a_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc((void*)G.x_hi, (short)0, (int)x_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rl =
        __builtin_amdgcn_make_buffer_rsrc((void*)(BF ? G.x_lo : G.x_hi), (short)0, (int)x_bytes, kBufferWord3);
    uint32_t va[2], vx[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t row = row0 + t * 32 + lr;
        va[t] = row < G.rows ? (uint32_t)(row * G.lda * EA) : a_bytes;      // rows beyond: 0
        vx[t] = (uint32_t)((col0 + t * 32 + lr) * G.ldx * EA);
    }

    f32x16 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[t][u][q] = 0.0f;

    u32x4 a_cur[2], h_cur[2], lo_cur[2], a_nxt[2], h_nxt[2], lo_nxt[2];
    auto load = [&](int64_t k, u32x4* a, u32x4* h, u32x4* lo) {
        const uint32_t ko = (uint32_t)((k + KL * lh) * EA);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            a[t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)(va[t] + ko), 0, 0));
            h[t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rh, (int)(vx[t] + ko), 0, 0));
            if constexpr (BF)
                lo[t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rl, (int)(vx[t] + ko), 0, 0));
        }
    };
    auto compute = [&](const u32x4* a, const u32x4* h, const u32x4* lo) {
        if constexpr (BF) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const bf16x8_t av = __builtin_bit_cast(bf16x8_t, a[t]);
                    acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, h[u]),
                                                                        acc[t][u], 0, 0, 0);
                    acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, lo[u]),
                                                                        acc[t][u], 0, 0, 0);
                }
        } else {
            // lane half lh holds k + 4 lh + q: the q-th product pairs k + q
            // (lanes 0-31) with k + 4 + q (lanes 32-63), the same in both operands
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[t][q]),
                                                                         __uint_as_float(h[u][q]), acc[t][u], 0, 0, 0);
        }
    };

    if (k_begin < k_end) {
        load(k_begin, a_cur, h_cur, lo_cur);
        for (int64_t k = k_begin; k < k_end; k += STEP) {
            const bool more = k + STEP < k_end;
            if (more) load(k + STEP, a_nxt, h_nxt, lo_nxt);
            compute(a_cur, h_cur, lo_cur);
            if (more) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    a_cur[t] = a_nxt[t];
                    h_cur[t] = h_nxt[t];
                    lo_cur[t] = lo_nxt[t];
                }
            }
        }
    }

    // acc[t][u][q]: row 8 (q/4) + 4 lh + q%4 of tile t, right-hand side lr of tile u.
    const int split = (int)blockIdx.z;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t i0 = row0 + t * 32 + 8 * g + 4 * lh;
                const int64_t r = col0 + u * 32 + lr;
                f32x4 v = {acc[t][u][4 * g], acc[t][u][4 * g + 1], acc[t][u][4 * g + 2], acc[t][u][4 * g + 3]};
                __builtin_nontemporal_store(v, (f32x4*)(G.part + mpart_index(r, i0, split, G.ld_part, G.splits)));
            }
}

// Tile of this workgroup.  Workgroups are dispatched round-robin over the
// 8 XCDs (linear id mod 8), so the linear id is remapped to make each XCD
// run a contiguous range of tiles: the two column tiles of a row tile and
// neighbouring row tiles of a k-chunk, which share operand rows, then meet
// in the same L2.
struct TileIdx {
    uint32_t x, y, z;
};
__device__ __forceinline__ TileIdx xcd_tile() {
    const uint32_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    const uint32_t total = gx * gy * gz;
    const uint32_t id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t L = (total % 8 == 0) ? (id % 8) * (total / 8) + id / 8 : id;
    return TileIdx{L % gx, (L / gx) % gy, L / (gx * gy)};
}

// Partial sums of a wave's MT x NT tiles of 32 x 32 (acc[t][u][q]: row
// 8 (q/4) + 4 lh + q%4 of tile t, right-hand side lr of tile u) leave through
// the wave's own LDS region (32 x 36 floats, free after the main loop's last
// barrier): written as [r][i], read back so that 8 lanes store one 128-byte
// run of the partial layout: whole lines instead of 16-byte pieces.
template <int MT, int NT>
__device__ __forceinline__ void store_partials_via_lds(const f32x16 (&acc)[MT][NT], float* wl, const MGemm& G,
                                                       int split, int64_t row0, int64_t col0, int l) {
    const int lr = l & 31, lh = l >> 5;
    const int rr = l >> 3, rc = 4 * (l & 7);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                f32x4 v = {acc[t][u][4 * g], acc[t][u][4 * g + 1], acc[t][u][4 * g + 2], acc[t][u][4 * g + 3]};
                *(f32x4*)(wl + lr * 36 + 8 * g + 4 * lh) = v;
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 8 * j + rr;
                const f32x4 v = *(const f32x4*)(wl + r * 36 + rc);
                __builtin_nontemporal_store(
                    v, (f32x4*)(G.part + mpart_index(col0 + u * 32 + r, row0 + t * 32 + rc, split, G.ld_part, G.splits)));
            }
            __builtin_amdgcn_wave_barrier();
        }
}

// Same product with the workgroup's operand tiles staged through LDS
// (double-buffered, one barrier per stage): each A row and each
// right-hand side is fetched from memory once per workgroup and read by
// the two waves that need it from LDS.  Stage: BK = 32 (BF16) or 16 (FP32)
// values of k, i.e. 64 bytes per row; LDS rows are padded to 80 bytes so
// the 16-byte fragment reads of 32 consecutive rows hit distinct banks.
template <bool BF>
__global__ __launch_bounds__(256) void mgemm_lds_kernel(MGemm G) {
    constexpr int EA = BF ? 2 : 4;
    constexpr int BK = 64 / EA;                 // k per stage
    constexpr int ROWB = 80;                    // LDS bytes per staged row
    constexpr int NPL = BF ? 2 : 1;             // right-hand-side planes
    constexpr int A_BYTES = kMTileRows * ROWB;
    constexpr int X_BYTES = kMTileCols * ROWB;
    constexpr int STAGE = A_BYTES + NPL * X_BYTES;
    __shared__ __align__(16) unsigned char lds[2 * STAGE];

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int lr = l & 31;
    const int lh = l >> 5;
    const int wm = w & 1, wn = w >> 1;
    const TileIdx ti = xcd_tile();
    const int64_t tile_r = (int64_t)ti.y * kMTileRows;
    const int64_t tile_c = (int64_t)ti.x * kMTileCols;
    const int64_t k_begin = (int64_t)ti.z * G.kchunk;
    int64_t k_end = k_begin + G.kchunk;
    if (k_end > G.kdim_pad) k_end = G.kdim_pad;

    const uint32_t a_bytes = (uint32_t)(G.rows * G.lda * EA);
    const uint32_t x_bytes = (uint32_t)(G.r_pad * G.ldx * EA);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void*)G.A, (short)0, (int)a_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rx0 = __builtin_amdgcn_make_buffer_rsrc((void*)G.x_hi, (short)0, (int)x_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rx1 =
        __builtin_amdgcn_make_buffer_rsrc((void*)(BF ? G.x_lo : G.x_hi), (short)0, (int)x_bytes, kBufferWord3);

    // Staging map: 16-byte chunk c of a stage = row c/4, bytes 16 (c%4).
    // A: 512 chunks (2 per thread); X: 512 per plane (2 per thread per plane).
    uint32_t ga[2], gx[2];
    int la[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = tid + 256 * q;
        const int row = c >> 2, kc = c & 3;
        const int64_t grow = tile_r + row;
        ga[q] = grow < G.rows ? (uint32_t)(grow * G.lda * EA + kc * 16) : a_bytes;
        gx[q] = (uint32_t)((tile_c + row) * G.ldx * EA + kc * 16);
        la[q] = row * ROWB + kc * 16;
    }
    u32x4 pa[2], px[NPL][2];
    auto fetch = [&](int64_t k) {
        const uint32_t ko = (uint32_t)(k * EA);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            pa[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)(ga[q] + ko), 0, 0));
            px[0][q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rx0, (int)(gx[q] + ko), 0, 0));
            if constexpr (BF)
                px[NPL - 1][q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rx1, (int)(gx[q] + ko), 0, 0));
        }
    };
    auto stash = [&](int buf) {
        unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            *(u32x4*)(base + la[q]) = pa[q];
#pragma unroll
            for (int p = 0; p < NPL; ++p) *(u32x4*)(base + A_BYTES + p * X_BYTES + la[q]) = px[p][q];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[t][u][q] = 0.0f;

    auto compute = [&](int buf) {
        const unsigned char* base = lds + buf * STAGE;
        // two MFMA k-steps per stage: 16 values (BF16) or 8 (FP32, 4 per lane half)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kb = ks * 32 + lh * 16;          // byte offset of the lane's k values in the row
            u32x4 af[2], xf[NPL][2];
#pragma unroll
            for (int t = 0; t < 2; ++t) af[t] = *(const u32x4*)(base + (wm * 64 + t * 32 + lr) * ROWB + kb);
#pragma unroll
            for (int p = 0; p < NPL; ++p)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    xf[p][u] = *(const u32x4*)(base + A_BYTES + p * X_BYTES + (wn * 64 + u * 32 + lr) * ROWB + kb);
            if constexpr (BF) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const bf16x8_t av = __builtin_bit_cast(bf16x8_t, af[t]);
                        acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, xf[0][u]),
                                                                            acc[t][u], 0, 0, 0);
                        acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            av, __builtin_bit_cast(bf16x8_t, xf[NPL - 1][u]), acc[t][u], 0, 0, 0);
                    }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
                            acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                __uint_as_float(af[t][q]), __uint_as_float(xf[0][u][q]), acc[t][u], 0, 0, 0);
            }
        }
    };

    const int nst = (int)((k_end - k_begin + BK - 1) / BK);
    if (nst > 0) {
        fetch(k_begin);
        stash(0);
        __syncthreads();
    }
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        const bool more = st + 1 < nst;
        if (more) fetch(k_begin + (int64_t)(st + 1) * BK);
        compute(buf);
        if (more) stash(buf ^ 1);
        __syncthreads();
    }

    static_assert(2 * STAGE >= 4 * 32 * 36 * 4, "epilogue regions must fit in the staging LDS");
    store_partials_via_lds<2, 2>(acc, (float*)lds + w * (32 * 36), G, (int)ti.z, tile_r + wm * 64, tile_c + wn * 64, l);
}

__device__ __forceinline__ int lds_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// BF16 form, tile staged through LDS with a deeper fetch pipeline: TR x TC
// tile per workgroup, each wave owning MT x NT tiles of 32 x 32, so one A
// fragment read from LDS feeds 2 NT matrix-core products and one
// right-hand-side fragment MT of them.  K streams from HBM with rows 16 KiB
// apart, so each workgroup keeps PD stages of loads in flight in registers
// (a ring; loads of a stage are issued PD - 1 stages before it is staged, and
// the ring holds A and both right-hand-side planes so that the in-order wait
// for one stage never waits for a later one), with two LDS buffers.
// 256 x 256 (one workgroup per CU, 96 KiB of LDS): per stage of 32 k values
// each of the four waves issues 64 products (2048 cycles of its SIMD's matrix
// core) against 96 KiB of LDS fragment reads and 48 KiB of staging writes,
// and K is fetched once per product (the tile spans 256 right-hand sides).
template <int WR, int WC, int MT, int NT, int PD>
__global__ __launch_bounds__(64 * WR * WC) void mgemm_ring_kernel(MGemm G) {
    constexpr int NTHR = 64 * WR * WC;
    constexpr int TR = WR * MT * 32;            // rows of A per workgroup
    constexpr int TC = WC * NT * 32;            // right-hand sides per workgroup
    constexpr int BK = 32;                      // k per stage (64 bytes per row)
    constexpr int A_BYTES = TR * 64;            // LDS: 64-byte rows, 16-byte chunks swizzled
    constexpr int X_BYTES = TC * 64;
    constexpr int STAGE = A_BYTES + 2 * X_BYTES;
    constexpr int CA = TR * 4 / NTHR;           // 16-byte A chunks per thread per stage
    constexpr int CX = TC * 4 / NTHR;           // chunks per right-hand-side plane per thread
    static_assert(TR * 4 % NTHR == 0 && TC * 4 % NTHR == 0, "staging map must cover the tile");
    static_assert(PD >= 1, "at least one stage in flight");
    extern __shared__ __align__(16) unsigned char lds[];

    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int w = tid >> 6;
    const int lr = l & 31;
    const int lh = l >> 5;
    const int wm = w % WR, wn = w / WR;
    const TileIdx ti = xcd_tile();
    const int64_t tile_r = (int64_t)ti.y * TR;
    const int64_t tile_c = (int64_t)ti.x * TC;
    const int64_t k_begin = (int64_t)ti.z * G.kchunk;
    int64_t k_end = k_begin + G.kchunk;
    if (k_end > G.kdim_pad) k_end = G.kdim_pad;

    // A plain (row-major, lda) or tiled (launch_mpack: a stage of the tile is
    // TR x 64 contiguous bytes, the next stage 16 KiB further)
    const bool blk = G.blocked != 0;
    const uint32_t a_bytes = blk ? (uint32_t)(G.rows_pad * G.kdim_pad * 2) : (uint32_t)(G.rows * G.lda * 2);
    const uint32_t a_kstep = blk ? (uint32_t)(kMPackRows * 64) : 64u;      // bytes per 32 values of k
    const uint32_t x_bytes = (uint32_t)(G.r_pad * G.ldx * 2);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void*)G.A, (short)0, (int)a_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc((void*)G.x_hi, (short)0, (int)x_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc((void*)G.x_lo, (short)0, (int)x_bytes, kBufferWord3);
    const int64_t a_tile = (tile_r / kMPackRows) * (G.kdim_pad / kMPackK) * (kMPackRows * 64) + (tile_r % kMPackRows) * 64;

    // Staging map: chunk c of a stage = row c/4, bytes 16 (c%4) of the row's 64.
    // In LDS, chunk kc of row r sits at slot kc ^ swz(r) of the row, with
    // swz(r) = ((r >> 1) ^ (r >> 2)) & 3: the 16-byte fragment reads (32
    // consecutive rows, one chunk) and the staging writes (4 chunks of
    // consecutive rows) then touch distinct banks in every group of 8 or 16
    // lanes, with no padding.
    uint32_t ga[CA], gx[CX];
    int la[CA], lx[CX];
#pragma unroll
    for (int q = 0; q < CA; ++q) {
        const int c = tid + NTHR * q;
        const int row = c >> 2, kc = c & 3;
        const int64_t grow = tile_r + row;
        if (blk)
            ga[q] = (uint32_t)(a_tile + c * 16);                                        // rows beyond are 0
        else
            ga[q] = grow < G.rows ? (uint32_t)(grow * G.lda * 2 + kc * 16) : a_bytes;     // rows beyond: 0
        la[q] = row * 64 + ((kc ^ lds_swz(row)) << 4);
    }
#pragma unroll
    for (int q = 0; q < CX; ++q) {
        const int c = tid + NTHR * q;
        const int row = c >> 2, kc = c & 3;
        gx[q] = (uint32_t)((tile_c + row) * G.ldx * 2 + kc * 16);
        lx[q] = row * 64 + ((kc ^ lds_swz(row)) << 4);
    }
    u32x4 pa[PD][CA], ph[PD][CX], pl[PD][CX];
    auto fetch = [&](int64_t k, int slot) {
        const uint32_t ko = (uint32_t)(k * 2);
        const uint32_t ka = (uint32_t)(k / 32) * a_kstep;
#pragma unroll
        for (int q = 0; q < CA; ++q)
            pa[slot][q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)(ga[q] + ka), 0, 0));
#pragma unroll
        for (int q = 0; q < CX; ++q) {
            ph[slot][q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rh, (int)(gx[q] + ko), 0, 0));
            pl[slot][q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rl, (int)(gx[q] + ko), 0, 0));
        }
    };
    auto stash = [&](int buf, int slot) {
        unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int q = 0; q < CA; ++q) *(u32x4*)(base + la[q]) = pa[slot][q];
#pragma unroll
        for (int q = 0; q < CX; ++q) {
            *(u32x4*)(base + A_BYTES + lx[q]) = ph[slot][q];
            *(u32x4*)(base + A_BYTES + X_BYTES + lx[q]) = pl[slot][q];
        }
    };

    f32x16 acc[MT][NT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[t][u][q] = 0.0f;

    // rows read by this lane are lr mod 32, so their swizzle is lds_swz(lr)
    const int kslot[2] = {(lh ^ lds_swz(lr)) << 4, ((2 + lh) ^ lds_swz(lr)) << 4};
    auto compute = [&](int buf) {
        const unsigned char* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kb = kslot[ks];                  // swizzled slot of the lane's 8 k values in the row
            u32x4 af[MT], hf[NT], lf[NT];
#pragma unroll
            for (int t = 0; t < MT; ++t) af[t] = *(const u32x4*)(base + (wm * MT * 32 + t * 32 + lr) * 64 + kb);
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int off = A_BYTES + (wn * NT * 32 + u * 32 + lr) * 64 + kb;
                hf[u] = *(const u32x4*)(base + off);
                lf[u] = *(const u32x4*)(base + off + X_BYTES);
            }
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    const bf16x8_t av = __builtin_bit_cast(bf16x8_t, af[t]);
                    acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, hf[u]),
                                                                        acc[t][u], 0, 0, 0);
                    acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, lf[u]),
                                                                        acc[t][u], 0, 0, 0);
                }
        }
    };

    // Stage s lives in ring slot s % PD from its fetch until it is staged
    // into LDS buffer s % 2 at the end of stage s - 1.  Fetches past the
    // last stage re-read the last stage (cache hits, never used), so every
    // fetch is unconditional and the wait before staging a stage leaves the
    // PD - 1 later stages in flight; the staging after the last stage writes
    // the idle buffer.
    const int nst = (int)((k_end - k_begin + BK - 1) / BK);
    const int64_t k_last = k_begin + (int64_t)(nst - 1) * BK;
    auto fetch_stage = [&](int s, int slot) {
        const int64_t k = k_begin + (int64_t)s * BK;
        fetch(k < k_last ? k : k_last, slot);
    };
    if (nst > 0) {
#pragma unroll
        for (int p = 0; p < PD; ++p) fetch_stage(p, p);
        stash(0, 0);
        __syncthreads();
        int st0 = 0;
        for (; st0 + PD <= nst; st0 += PD) {
#pragma unroll
            for (int j = 0; j < PD; ++j) {
                const int st = st0 + j;         // stage computed now; its slot j is free again
                fetch_stage(st + PD, j);
                compute(st & 1);
                stash((st + 1) & 1, (j + 1) % PD);
                __syncthreads();
            }
        }
#pragma unroll
        for (int j = 0; j < PD - 1; ++j) {
            const int st = st0 + j;
            if (st < nst) {
                compute(st & 1);
                stash((st + 1) & 1, (j + 1) % PD);
                __syncthreads();
            }
        }
    }

    static_assert(2 * STAGE >= NTHR / 64 * 32 * 36 * 4, "epilogue regions must fit in the staging LDS");
    store_partials_via_lds<MT, NT>(acc, (float*)lds + w * (32 * 36), G, (int)ti.z, tile_r + wm * MT * 32,
                                   tile_c + wn * NT * 32, l);
}

template <bool TRANS>
__global__ __launch_bounds__(256) void mpack_kernel(const uint16_t* __restrict__ src, int64_t ld, int64_t src_rows,
                                                    int64_t src_cols, uint16_t* __restrict__ dst, int64_t rows_pad,
                                                    int64_t kdim_pad) {
    const int64_t kb_count = kdim_pad / kMPackK;
    const int64_t total = rows_pad * kdim_pad / 8;              // 16-byte chunks of dst
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
        const int64_t blk = c / (kMPackRows * 4);
        const int64_t w = c % (kMPackRows * 4);
        const int64_t row = (blk / kb_count) * kMPackRows + w / 4;
        const int64_t k0 = (blk % kb_count) * kMPackK + (w % 4) * 8;
        uint16_t v[8];
        if (!TRANS && row < src_rows && k0 + 8 <= src_cols) {
            const u32x4 x = *(const u32x4*)(src + row * ld + k0);
            *(u32x4*)(dst + c * 8) = x;
            continue;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t k = k0 + e;
            const bool ok = TRANS ? (k < src_rows && row < src_cols) : (row < src_rows && k < src_cols);
            v[e] = ok ? (TRANS ? src[k * ld + row] : src[row * ld + k]) : (uint16_t)0;
        }
        u32x4 y = {(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                   (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)};
        *(u32x4*)(dst + c * 8) = y;
    }
}

// q^fi for the BF16 form, whose right-hand sides keep ~16 bits: log2 of the
// mantissa and exp2 of the fractional exponent on the FP32 units (relative
// error ~3e-7), exponent handling in FP64 so the full FP64 range is kept.
// q must be positive and finite.
__device__ __forceinline__ double pow_bf16_form(double q, double fi) {
    int e;
    const double mt = frexp(q, &e);                                   // [0.5, 1)
    const double t = fi * ((double)e + (double)__builtin_amdgcn_logf((float)mt));
    const double ti = floor(t);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(t - ti)), (int)ti);
}

// Workgroup: 1024 consecutive rows of right-hand side r = blockIdx.y; lane
// t of the workgroup takes rows t, t + 256, t + 512, t + 768 of the block, so
// every load and store of the workgroup is one contiguous run per wave.
// Workgroup: 1024 consecutive rows of right-hand side r = blockIdx.y; lane
// t of the workgroup takes rows t, t + 256, t + 512, t + 768 of the block.
// The chunk sums of 32 consecutive rows sit side by side (mpart_index), so a
// wave's partial reads for all chunks form one contiguous run.
__global__ __launch_bounds__(256) void mepi_kernel(MEpi E) {
    const int64_t r = blockIdx.y;
    const int64_t ib = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint32_t fl = 0;
    double tg[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = ib + 256 * e;
        tg[e] = (E.mode == 0 && r < E.R && i < E.rows) ? E.target[r * E.rows + i] : 0.0;
    }
    const float* pp[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = ib + 256 * e;
        pp[e] = E.part + mpart_index(r, i < E.ld_next ? i : 0, 0, E.ld_part, E.splits);
    }
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    int s = 0;
    for (; s + 4 <= E.splits; s += 4) {            // chunks added in ascending order
        float p[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) p[q][e] = pp[e][(s + q) * 32];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) S[e] += (double)p[q][e];
    }
    for (; s < E.splits; ++s) {
#pragma unroll
        for (int e = 0; e < 4; ++e) S[e] += (double)pp[e][s * 32];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = ib + 256 * e;
        if (i >= E.ld_next) break;
        const bool valid = r < E.R && i < E.rows;
        const double sm = S[e] * E.k_scale;
        double y = 0.0;
        if (valid) {
            const int64_t o = r * E.rows + i;
            if (E.mode == 0) {
                const double tgt = tg[e];
                const double q = tgt / sm;
                if (E.bf16 && !E.fi_is_one && q > 0.0 && isfinite(q))
                    y = pow_bf16_form(q, E.fi);
                else
                    y = scale_factor(tgt, sm, E.fi, E.fi_is_one, 0.0);
                if (tgt > 0.0 && !(sm > 0.0)) fl |= UOT_FLAG_ZERO_SUM;
                if (!isfinite(y)) fl |= UOT_FLAG_NONFINITE;
                if (E.store_y) E.y[o] = y;
                if (E.marg) E.marg[o] = y * sm;
            } else {
                E.marg[o] = E.y[o] * sm;
            }
        }
        if (E.mode == 0) {
            const int64_t o = r * E.ld_next + i;      // next right-hand sides, zero padding
            if (E.bf16) {
                const uint16_t hi = f64_to_bf16(y);
                const double h = (double)__uint_as_float((uint32_t)hi << 16);
                ((uint16_t*)E.next_hi)[o] = hi;
                ((uint16_t*)E.next_lo)[o] = f64_to_bf16(y - h);
            } else {
                ((float*)E.next_hi)[o] = (float)y;
            }
        }
    }
    if (fl) atomicOr(E.flags, fl);
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ K, int64_t ldk, int64_t n, int64_t m,
                                                        T* __restrict__ KT, int64_t ldkt) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 32 x 8
    for (int64_t bj = blockIdx.x; bj * 32 < m; bj += gridDim.x)
        for (int64_t bi = blockIdx.y; bi * 32 < ldkt; bi += gridDim.y) {
            for (int k = ty; k < 32; k += 8) {
                const int64_t i = bi * 32 + k, j = bj * 32 + tx;
                tile[k][tx] = (i < n && j < m) ? K[i * ldk + j] : T(0);
            }
            __syncthreads();
            for (int k = ty; k < 32; k += 8) {
                const int64_t j = bj * 32 + k, i = bi * 32 + tx;
                if (j < m && i < ldkt) KT[j * ldkt + i] = tile[tx][k];
            }
            __syncthreads();
        }
}

__global__ void ones_rhs_kernel(int bf16, uint16_t* hi16, uint16_t* lo16, float* f, int64_t R, int64_t r_pad,
                                int64_t m, int64_t ld) {
    const int64_t total = r_pad * ld;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int64_t r = idx / ld, j = idx % ld;
        const bool one = r < R && j < m;
        if (bf16) {
            hi16[idx] = one ? (uint16_t)0x3f80u : (uint16_t)0;
            lo16[idx] = 0;
        } else {
            f[idx] = one ? 1.0f : 0.0f;
        }
    }
}

__device__ __forceinline__ double kl_term_m(double x, double y) {
    if (x > 0.0) return x * log(x / y) - x + y;
    return y;
}

__device__ double block_sum_256(double x, double* sh) {
    x = wave_sum_f64(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(256) void multi_loss_kernel(const double* U, const double* V, const double* Rm,
                                                         const double* Cm, const double* A, const double* B, int64_t n,
                                                         int64_t m, double eps, double tau, int fi_is_one,
                                                         double* losses, uint32_t* flags) {
    __shared__ double sh[4];
    const int64_t r = blockIdx.x;
    double rlu = 0.0, rs = 0.0, klr = 0.0, clv = 0.0, klc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double ri = Rm[r * n + i];
        if (ri > 0.0) rlu += ri * log(U[r * n + i]);
        rs += ri;
        klr += kl_term_m(ri, A[r * n + i]);
    }
    for (int64_t j = threadIdx.x; j < m; j += 256) {
        const double cj = Cm[r * m + j];
        if (cj > 0.0) clv += cj * log(V[r * m + j]);
        klc += kl_term_m(cj, B[r * m + j]);
    }
    rlu = block_sum_256(rlu, sh);
    rs = block_sum_256(rs, sh);
    clv = block_sum_256(clv, sh);
    double L = eps * (rlu + clv - rs);
    if (!fi_is_one) {
        klr = block_sum_256(klr, sh);
        klc = block_sum_256(klc, sh);
        L += tau * (klr + klc);
    }
    if (threadIdx.x == 0) {
        losses[r] = L;
        if (!isfinite(L)) atomicOr(flags, UOT_FLAG_NONFINITE);
    }
}

__global__ void multi_info_kernel(uot_info* info, int64_t iters, uint32_t* flags, int reset) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (reset) {
        *flags = 0u;
        return;
    }
    info->iters = iters;
    info->err = 0.0;
    info->absorptions = 0;
    info->flags = *flags;
}

}  // namespace

hipError_t launch_multi_info(uot_info* info, int64_t iters, uint32_t* flags, int reset, hipStream_t stream) {
    hipLaunchKernelGGL(multi_info_kernel, dim3(1), dim3(64), 0, stream, info, iters, flags, reset);
    return hipGetLastError();
}

template <int WR, int WC, int MT, int NT, int PD>
static hipError_t launch_ring(const MGemm& G, hipStream_t stream) {
    constexpr int TR = WR * MT * 32, TC = WC * NT * 32;
    constexpr int lds = 2 * (TR + 2 * TC) * 64;
    if (G.r_pad % TC != 0 || G.rows_pad % TR != 0) return hipErrorInvalidValue;
    auto fn = mgemm_ring_kernel<WR, WC, MT, NT, PD>;
    if (lds > 65536) {      // on every call: the limit is per device, and callers may use several
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)(G.r_pad / TC), (unsigned)(G.rows_pad / TR), (unsigned)G.splits);
    hipLaunchKernelGGL(fn, grid, dim3(64 * WR * WC), lds, stream, G);
    return hipGetLastError();
}

hipError_t launch_mgemm(int bf16, const MGemm& G, hipStream_t stream) {
    if (G.variant >= 3) {
        if (!bf16) return hipErrorInvalidValue;
        switch (G.variant) {
            case 3: return launch_ring<2, 4, 4, 2, 3>(G, stream);
            case 4: return launch_ring<2, 2, 2, 2, 4>(G, stream);
            default: return hipErrorInvalidValue;
        }
    }
    dim3 grid((unsigned)(G.r_pad / kMTileCols), (unsigned)(G.rows_pad / kMTileRows), (unsigned)G.splits);
    if (G.variant == 1) {
        if (bf16)
            hipLaunchKernelGGL(mgemm_lds_kernel<true>, grid, dim3(256), 0, stream, G);
        else
            hipLaunchKernelGGL(mgemm_lds_kernel<false>, grid, dim3(256), 0, stream, G);
    } else {
        if (bf16)
            hipLaunchKernelGGL(mgemm_kernel<true>, grid, dim3(256), 0, stream, G);
        else
            hipLaunchKernelGGL(mgemm_kernel<false>, grid, dim3(256), 0, stream, G);
    }
    return hipGetLastError();
}

hipError_t launch_mepi(const MEpi& E, hipStream_t stream) {
    if (E.r_pad > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((E.ld_next + 1023) / 1024), (unsigned)E.r_pad);
    hipLaunchKernelGGL(mepi_kernel, grid, dim3(256), 0, stream, E);
    return hipGetLastError();
}

hipError_t launch_transpose(int k_dtype, const void* K, int64_t ldk, int64_t n, int64_t m, void* KT, int64_t ldkt,
                            hipStream_t stream) {
    dim3 grid((unsigned)std::min<int64_t>((m + 31) / 32, 1024), (unsigned)std::min<int64_t>((ldkt + 31) / 32, 1024));
    switch (k_dtype) {
        case UOT_F64: hipLaunchKernelGGL(transpose_kernel<uint64_t>, grid, dim3(256), 0, stream, (const uint64_t*)K, ldk, n, m, (uint64_t*)KT, ldkt); break;
        case UOT_F32: hipLaunchKernelGGL(transpose_kernel<uint32_t>, grid, dim3(256), 0, stream, (const uint32_t*)K, ldk, n, m, (uint32_t*)KT, ldkt); break;
        case UOT_BF16: hipLaunchKernelGGL(transpose_kernel<uint16_t>, grid, dim3(256), 0, stream, (const uint16_t*)K, ldk, n, m, (uint16_t*)KT, ldkt); break;
        case UOT_FP8_E4M3: hipLaunchKernelGGL(transpose_kernel<uint8_t>, grid, dim3(256), 0, stream, (const uint8_t*)K, ldk, n, m, (uint8_t*)KT, ldkt); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mpack(int trans, const void* src, int64_t ld, int64_t src_rows, int64_t src_cols, void* dst,
                        int64_t rows_pad, int64_t kdim_pad, hipStream_t stream) {
    if (rows_pad % kMPackRows != 0 || kdim_pad % kMPackK != 0) return hipErrorInvalidValue;
    int64_t blocks = (rows_pad * kdim_pad / 8 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (trans)
        hipLaunchKernelGGL(mpack_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint16_t*)src, ld,
                           src_rows, src_cols, (uint16_t*)dst, rows_pad, kdim_pad);
    else
        hipLaunchKernelGGL(mpack_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint16_t*)src, ld,
                           src_rows, src_cols, (uint16_t*)dst, rows_pad, kdim_pad);
    return hipGetLastError();
}

hipError_t launch_ones_rhs(int bf16, void* hi, void* lo, int64_t R, int64_t r_pad, int64_t m, int64_t ld,
                           hipStream_t stream) {
    int64_t blocks = (r_pad * ld + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ones_rhs_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, bf16, (uint16_t*)hi,
                       (uint16_t*)lo, (float*)hi, R, r_pad, m, ld);
    return hipGetLastError();
}

hipError_t launch_multi_loss(const double* U, const double* V, const double* Rm, const double* Cm, const double* A,
                             const double* B, int64_t n, int64_t m, int64_t R, double eps, double tau, int fi_is_one,
                             double* losses, uint32_t* flags, hipStream_t stream) {
    hipLaunchKernelGGL(multi_loss_kernel, dim3((unsigned)R), dim3(256), 0, stream, U, V, Rm, Cm, A, B, n, m, eps, tau,
                       fi_is_one, losses, flags);
    return hipGetLastError();
}

}  // namespace uot
