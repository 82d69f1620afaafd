// Internal declarations shared by the HIP translation units of libuot.so.
// (Not part of the public C-ABI; see include/uot.h.)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uot.h"

namespace uot {

// ---------------------------------------------------------------------------
// Device control block (lives in the workspace).
// ---------------------------------------------------------------------------
struct Ctrl {
    uint32_t done;      // set once the stopping test passed; later launches return at once
    uint32_t bar;       // grid-barrier arrival count of the persistent kernel
    uint32_t flags;     // UOT_FLAG_* accumulated on the device
    uint32_t pad0;
    int64_t iters;      // iteration at which the stopping test passed (valid when done)
    double err;         // its error (valid when done)
};

// ---------------------------------------------------------------------------
// Storage types of K and their 16-byte vector loads.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
struct fp8_t { uint8_t bits; };

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename KT> struct KVec;
template <> struct KVec<double> { using raw = f64x2; static constexpr int N = 2; };
template <> struct KVec<float>  { using raw = f32x4; static constexpr int N = 4; };
template <> struct KVec<bf16_t> { using raw = u32x4; static constexpr int N = 8; };
template <> struct KVec<fp8_t>  { using raw = u32x4; static constexpr int N = 16; };

template <typename T>
__device__ __forceinline__ T zero_raw() {
    T z;
    __builtin_memset(&z, 0, sizeof(T));
    return z;
}

// Expand one 16-byte vector of stored K into N arithmetic values.
template <typename KT, typename AT> struct Unpack;
template <typename AT> struct Unpack<double, AT> {
    static __device__ __forceinline__ void run(const f64x2& r, AT* o) {
        o[0] = (AT)r[0];
        o[1] = (AT)r[1];
    }
};
template <typename AT> struct Unpack<float, AT> {
    static __device__ __forceinline__ void run(const f32x4& r, AT* o) {
        o[0] = (AT)r[0];
        o[1] = (AT)r[1];
        o[2] = (AT)r[2];
        o[3] = (AT)r[3];
    }
};
// bfloat16: the upper 16 bits of an FP32 value.
template <typename AT> struct Unpack<bf16_t, AT> {
    static __device__ __forceinline__ void run(const u32x4& r, AT* o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (AT)__uint_as_float(r[q] << 16);
            o[2 * q + 1] = (AT)__uint_as_float(r[q] & 0xffff0000u);
        }
    }
};
// OCP E4M3FN through the gfx950 packed conversion (two values per instruction).
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename AT> struct Unpack<fp8_t, AT> {
    static __device__ __forceinline__ void run(const u32x4& r, AT* o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)r[q], false);
            f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)r[q], true);
            o[4 * q] = (AT)lo[0];
            o[4 * q + 1] = (AT)lo[1];
            o[4 * q + 2] = (AT)hi[0];
            o[4 * q + 3] = (AT)hi[1];
        }
    }
};

// FP64 -> bfloat16, round to nearest even: truncate to FP32 and mark
// inexactness in the last FP32 bit (round to odd), then round the FP32 bits
// to 16 (FP32 keeps 16 more mantissa bits, so no double rounding occurs).
// Finite inputs only; results below the normal range are flushed to zero.
__device__ __forceinline__ uint16_t f64_to_bf16(double d) {
    float f = __double2float_rz(d);
    uint32_t u = __float_as_uint(f);
    if ((double)f != d) u |= 1u;
    if ((u & 0x7f800000u) == 0) return (uint16_t)((u >> 16) & 0x8000u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP64 x >= 0 -> OCP E4M3FN (bias 7, max 448, subnormals 2^-9 .. 7 * 2^-9),
// round to nearest even, saturating at 448.
__device__ __forceinline__ uint8_t f64_to_e4m3(double x) {
    if (!(x > 0.0)) return 0;
    if (x >= 448.0) return 0x7e;
    int e;
    (void)frexp(x, &e);      // x = f * 2^e, f in [0.5, 1): floor(log2 x) = e - 1
    int ex = e - 1;
    if (ex < -6) {            // subnormal: multiples of 2^-9
        double q = rint(ldexp(x, 9));
        return (uint8_t)q;    // q = 8 is the smallest normal's code (0x08)
    }
    double mant = rint(ldexp(x, 3 - ex));   // in [8, 16]
    if (mant >= 16.0) {
        mant = 8.0;
        ex += 1;
    }
    if (ex > 8) return 0x7e;
    int code = ((ex + 7) << 3) | ((int)mant - 8);
    if (code > 0x7e) code = 0x7e;
    return (uint8_t)code;
}

// Four adjacent column partials (one 16-byte FP32 chunk or two FP64 chunks)
// widened to FP64.
template <typename AT> struct Chunk4;
template <> struct Chunk4<float> {
    static __device__ __forceinline__ void load(const float* p, double* o) {
        f32x4 x = *(const f32x4*)p;
        o[0] = x[0]; o[1] = x[1]; o[2] = x[2]; o[3] = x[3];
    }
};
template <> struct Chunk4<double> {
    static __device__ __forceinline__ void load(const double* p, double* o) {
        f64x2 x = *(const f64x2*)p;
        f64x2 y = *(const f64x2*)(p + 2);
        o[0] = x[0]; o[1] = x[1]; o[2] = y[0]; o[3] = y[1];
    }
};

// Bound on the sleep-loop iterations of one grid-barrier wait (about a
// second); exceeding it sets UOT_FLAG_BARRIER_TIMEOUT instead of hanging.
constexpr uint32_t kBarrierSpinLimit = 1u << 24;

// ---------------------------------------------------------------------------
// Cross-lane helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double x, int lane) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_readlane(lo, lane);
    hi = __builtin_amdgcn_readlane(hi, lane);
    return __hiloint2double(hi, lo);
}

// DPP move of a double (both halves with the same lane pattern).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave; every lane returns the same bits.
// Within each row of 16 lanes: partner exchanges (lane ^ 1, lane ^ 2 via
// quad permutes, then the half-row and row mirrors, which pair each lane with
// one holding the other 4- and 8-lane sum), so all 16 lanes of a row hold
// the row sum; the four row sums are then read from lanes 0, 16, 32, 48 and
// added in that order.  Must be called with all 64 lanes active.
__device__ __forceinline__ double wave_sum_f64(double x) {
    x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
    x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
    x += dpp_f64<0x141>(x);   // row_half_mirror
    x += dpp_f64<0x140>(x);   // row_mirror
    double r0 = readlane_f64(x, 0), r1 = readlane_f64(x, 16);
    double r2 = readlane_f64(x, 32), r3 = readlane_f64(x, 48);
    return ((r0 + r1) + r2) + r3;
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16), every lane of a
// group returning the same bits: the first log2(G) exchanges of wave_sum_f64.
template <int G>
__device__ __forceinline__ double group_sum_f64(double x) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1-16 lanes");
    if constexpr (G >= 2) x += dpp_f64<0xB1>(x);
    if constexpr (G >= 4) x += dpp_f64<0x4E>(x);
    if constexpr (G >= 8) x += dpp_f64<0x141>(x);
    if constexpr (G >= 16) x += dpp_f64<0x140>(x);
    return x;
}

__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ float readlane_f32(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

template <typename AT> __device__ __forceinline__ AT readlane_at(AT x, int lane);
template <> __device__ __forceinline__ float readlane_at<float>(float x, int lane) { return readlane_f32(x, lane); }
template <> __device__ __forceinline__ double readlane_at<double>(double x, int lane) { return readlane_f64(x, lane); }

// Scaling factor (target / sum)^fi times exp(shift); zero target -> 0.
__device__ __forceinline__ double scale_factor(double target, double sum, double fi, int fi_is_one,
                                               double shift) {
    if (target == 0.0) return 0.0;
    double q = target / sum;
    double f = fi_is_one ? q : exp(fi * log(q));
    if (shift != 0.0) f *= exp(shift);
    return f;
}

__device__ __forceinline__ uint32_t ld_volatile_u32(const uint32_t* p) {
    return *(const volatile uint32_t*)p;
}

// Relative L1 change of the column marginal from the per-block sums the
// column finalize wrote: sum_k bp[2k] / sum_k bp[2k+1].  Called by one full
// wave; lanes stride over blocks, then a butterfly, so every caller gets the
// same bits.
__device__ __forceinline__ double stop_error(const double* bp, int nblocks, int lane) {
    double dn = 0.0, dc = 0.0;
    for (int k = lane; k < nblocks; k += 64) {
        dn += bp[2 * k];
        dc += bp[2 * k + 1];
    }
    dn = wave_sum_f64(dn);
    dc = wave_sum_f64(dc);
    return dn / dc;
}

// ---------------------------------------------------------------------------
// Pass kernels (pass.hip).
// ---------------------------------------------------------------------------
// MODE_MATRIX: the paper's literal in-place form -- the fused pass with v
// holding the column factors, writing each row back multiplied by the column
// factors and its row factor, and accumulating the rescaled entries.
enum PassMode { MODE_FUSED = 0, MODE_ROW = 1, MODE_COL = 2, MODE_MARG = 3, MODE_MATRIX = 4 };

struct PassLaunch {
    const void* K;
    int64_t ldk;
    int64_t n, m;
    int64_t rows_per_wg;
    int32_t grid;              // number of row strips (workgroups)
    const double* v;           // m
    const double* a;           // n
    double* u;                 // n
    double* s_out;             // n (MODE_MARG: K v; MODE_MATRIX: row sums of the rescaled rows, if set)
    void* partials;            // grid x ldp, FP32 or FP64
    int64_t ldp;
    double fi;
    int32_t fi_is_one;
    const double* fpot;        // optional row potentials (stabilised form)
    double inv_eps;
    Ctrl* ctrl;
    int32_t check_done;        // 1: return at once when ctrl->done is set
    int64_t ldv_bytes;         // LDS bytes for v (shapes that keep v in LDS), multiple of 16
    // Stopping test of the previous iteration, evaluated at the start of this
    // one (the first pass of iteration `iter` reads the column-finalize block
    // sums of iteration iter-1): stop when tol > 0 and err <= tol.
    int64_t iter;              // 1-based index of the iteration this launch belongs to
    int32_t test_stop;         // 1 on the first pass of an iteration
    int32_t fin_blocks;
    const double* blockpart;   // 2 x fin_blocks: sum|c - c_prev|, sum|c| per block
    double tol;
    double* s_trace;           // optional (FUSED/ROW): row sums K v written per row
    double k_scale;            // K = k_scale * stored values (1 except FP8)
};

struct PassShape {
    int wg;       // threads per workgroup
    int nc;       // 16-byte chunks per lane per row
    int depth;    // rows (or row batches) in flight (software pipeline depth)
    int vlds;     // 1: v read from LDS, 0: v held in registers
    int rb;       // rows per barrier (batch size)
};

// Number of instantiated shapes and their table.
int pass_shape_count();
PassShape pass_shape(int idx);
size_t pass_lds_bytes(int shape_idx, int mode, int acc64, const PassLaunch& L);
// Workgroups of a pass instantiation that fit on one CU with `lds` bytes of
// dynamic LDS (0 on error).
int pass_resident_per_cu(int k_dtype, int acc64, int mode, int shape_idx, size_t lds);

// Launch one streaming pass; returns hipSuccess or an error.  k_dtype and
// acc64 select the instantiation; shape_idx indexes pass_shape().
// The in-place matrix form (MODE_MATRIX) on a one-row shape; FP32 or FP64 storage.
hipError_t launch_pass_matrix(int k_dtype, int shape_idx, const PassLaunch& L, hipStream_t stream);
hipError_t launch_pass(int k_dtype, int acc64, int mode, int shape_idx, const PassLaunch& L,
                       hipStream_t stream);

// ---------------------------------------------------------------------------
// Auxiliary kernels (aux.hip).
// ---------------------------------------------------------------------------
struct FinLaunch {
    const void* partials;     // G x ldp
    int64_t ldp;
    int32_t G;
    int64_t m;
    const double* b;
    double* v;                // in/out
    double* w_out;            // m (optional)
    double* cprev;            // m
    double* c_out;            // m (marginal mode, optional)
    double fi;
    int32_t fi_is_one;
    const double* gpot;       // optional column potentials
    double inv_eps;
    Ctrl* ctrl;
    double* blockpart;        // 2 x nblocks
    int32_t marginal_only;    // 1: only w and c are formed
    int32_t acc64;
    double k_scale;           // K = k_scale * stored values
};

hipError_t launch_finalize(const FinLaunch& F, hipStream_t stream);

// Persistent (cooperative) whole-loop launch of the fused pass.
struct PersistLaunch {
    PassLaunch L;             // L.fin_blocks = grid, L.blockpart: 2 x grid
    FinLaunch F;              // b, v, w_out, cprev, fi, gpot
    int32_t max_iter;
    int32_t fin_cols;         // columns finalized per workgroup (multiple of 4, <= workgroup size)
    int64_t scratch_bytes;    // LDS bytes before the row staging: max(v, finalize scratch)
};
// ---------------------------------------------------------------------------
// Adjoint kernels (adj.hip).
// ---------------------------------------------------------------------------
enum AdjPhase { ADJ_SEED = 0, ADJ_STEP = 1 };
struct AdjLaunch {
    const void* K;
    int64_t ldk;
    int64_t n, m;
    int64_t rows_per_wg;
    int32_t grid;
    const double* A;          // m: step: wbar_t; seed: cbar * v_T
    const double* B;          // m: step: v_{t-1}; seed: v_T
    const double* y;          // m x dim target points (dim > 0)
    const double* u;          // n: u_t (step) / u_T (seed)
    const double* s;          // n: s_t (step)
    const double* a;          // n
    double* useed;            // n: written by the seed pass, added at step T
    int32_t add_seed;
    double* abar;             // n
    double* gsum;             // n: sum_j dL/dC_ij
    double* gy;               // n x dim: sum_j dL/dC_ij y_j
    void* partials;           // grid x ldp (AT)
    int64_t ldp;
    double fi, eps, tau;
    int32_t tau_inf;
    // Factors of this pass's two rank-1 terms of Kbar, stored for the cost
    // gradient (NULL = not stored): step t adds u_t wbar_t^T + sbar_t v_{t-1}^T,
    // the seed (rbar u_T) v_T^T + u_T (cbar v_T)^T.
    double* st_q;             // n: the row factor the column partials use (step: sbar_t; seed: rbar u_T)
    double* st_u;             // n: u
    double* st_a;             // m: copy of A
    double* st_b;             // m: copy of B
};
size_t adj_lds_bytes(int64_t rows_per_wg, int dim, int64_t m, int elem);
int adj_chunks_max(int k_dtype);
int adj_wg();
hipError_t launch_adj(int k_dtype, int nc, int phase, int dim, const AdjLaunch& L, hipStream_t stream);

enum AdjColMode { ADJ_COL_PREP = 0, ADJ_COL_SEED = 1, ADJ_COL_STEP = 2 };
struct AdjColLaunch {
    const void* partials;
    int64_t ldp;
    int32_t G;
    int64_t m;
    int32_t mode;
    int32_t acc64;
    const double* v;          // v_t of the step (v_T for PREP/SEED)
    const double* b;
    double* w;                // PREP writes K^T u_T; others read w_t
    double* cbar;             // PREP writes, SEED reads
    double* bbar;             // PREP writes, others accumulate
    double* out;              // PREP: cbar * v; SEED/STEP: wbar for the next step
    double fi, eps, tau;
    int32_t tau_inf;
};
hipError_t launch_adj_col(const AdjColLaunch& C, hipStream_t stream);

struct AdjFinish {
    const double* grad_loss;
    const double* abar; const double* bbar; const double* gsum; const double* gy;
    const double* x;
    double* grad_a; double* grad_b; double* grad_x;
    int64_t n, m;
    int32_t dim;
};
hipError_t launch_adj_finish(const AdjFinish& F, hipStream_t stream);

// Cost gradient from the stored factors (adj.hip):
//   G_ij = scale K_ij sum_s Lf[s][i] Rf[s][j],  scale = -grad_loss / eps,
// a dense FP64 product on the matrix cores with the kernel applied in its
// epilogue; optionally the per-row-tile column sums of G and G x_i that give
// the target-point gradient.
constexpr int kGradcSlotPad = 16;    // factor slots padded to a multiple of this (zero factors)
constexpr int kGradcRowPad = 128;    // factor rows padded to a multiple of this (zero entries)
struct GradCLaunch {
    const void* K;            // stored kernel (FP32 or FP64), k_scale 1
    int32_t k_dtype;
    int64_t ldk;
    int64_t n, m;
    int64_t nterms;           // rank of Kbar (2T + 2), padded to kGradcSlotPad
    const double* Lf;         // nterms x ldl (ldl = n padded to kGradcRowPad)
    const double* Rf;         // nterms x ldr
    int64_t ldl, ldr;
    const double* grad_loss;  // device scalar
    double inv_eps;
    double* G;                // n x ldg, or NULL
    int64_t ldg;
    const double* x;          // n x dim source points (ysum != NULL)
    int32_t dim;
    double* ysum;             // row tiles x m x (1 + dim) column sums, or NULL
};
int gradc_row_tiles(int64_t n);
hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t stream);
hipError_t launch_gradc(const GradCLaunch& L, hipStream_t stream);
// Implicit (envelope) gradients from marginal passes (adj.hip).
hipError_t launch_env_weight(const double* u, const double* x, int64_t n, const double* v, const double* y, int64_t m,
                             int32_t dim, int32_t d, double* ud, double* vd, hipStream_t stream);
struct EnvFinish {
    const double* grad_loss;
    const double* u; const double* v; const double* a; const double* b;
    const double* s; const double* w;          // K v, K^T u
    const double* sy; const double* wx;        // dim x n: K (v y_d); dim x m: K^T (u x_d)
    const double* x; const double* y;
    double* grad_a; double* grad_b; double* grad_x; double* grad_y;
    int64_t n, m;
    int32_t dim;
    int32_t tau_inf;
    double tau;
};
hipError_t launch_env_finish(const EnvFinish& F, hipStream_t stream);
// grad_y[j][d] = 2 (y_jd sum_i G_ij - sum_i G_ij x_id), the sums taken over row tiles in order.
hipError_t launch_grady_finish(const double* ysum, int32_t tiles, const double* y, int64_t m, int32_t dim,
                               double* grad_y, hipStream_t stream);

// Largest co-resident grid for the shape (0 when the shape cannot run persistently).
int persist_max_grid(int k_dtype, int acc64, int shape_idx, size_t lds);
hipError_t launch_persist(int k_dtype, int acc64, int shape_idx, const PersistLaunch& P, size_t lds,
                          hipStream_t stream);
int finalize_blocks(int64_t m);

hipError_t launch_init(double* u, int64_t n, const double* u0, double* v, int64_t m, const double* v0,
                       double* cprev, Ctrl* ctrl, hipStream_t stream);

struct ObjLaunch {
    const double* u; const double* v;
    const double* s; const double* w;   // K v and K^T u
    const double* a; const double* b;
    int64_t n, m;
    double eps, tau;
    int32_t tau_inf;
    double* r_out; double* c_out; double* loss;
    uot_info* info;
    const Ctrl* ctrl;
    double tol;
    int64_t iters_run;        // iterations enqueued (used when the stopping test never passed)
    const double* blockpart;  // block sums of the last finalize (error when not stopped)
    int32_t fin_blocks;
    const double* fpot;       // optional row potentials: total scaling u * e^{f/eps}
    const double* gpot;       // optional column potentials
    double* f_out;            // optional eps log(total u)
    double* g_out;            // optional eps log(total v)
    double* u_tot;            // optional total u (may overflow to inf)
    double* v_tot;            // optional total v
    int32_t absorptions;      // absorptions performed (counted on the host)
    int32_t info_only;        // write info only (no marginals or objective)
};
hipError_t launch_objective(const ObjLaunch& O, hipStream_t stream);

// Stabilised kernel: f_i = min_j (C_ij - g_j), then g_j = min_i (C_ij - f_i),
// Kt_ij = store(scale exp((f_i + g_j - C_ij)/eps)); u and v rescaled so the
// totals u e^{f/eps}, v e^{g/eps} are unchanged.  gmin_scratch: m x 8 bytes.
hipError_t launch_rebuild(const double* C, int64_t ldc, int64_t n, int64_t m, double eps, double* f, double* g,
                          double* u, double* v, void* gmin_scratch, int k_dtype, void* K, int64_t ldk,
                          double store_scale, int first, hipStream_t stream);
// out[0] = max_i |log u_i| (u_i > 0), out[1] = max_j |log v_j| (v_j > 0).
hipError_t launch_absorb_check(const double* u, int64_t n, const double* v, int64_t m, double* out,
                               hipStream_t stream);
// g_j += eps log v_j, v_j = 1 (v_j > 0).
hipError_t launch_absorb_apply(double* v, double* g, int64_t m, double eps, hipStream_t stream);
// Decode stored K to FP32 as the passes read it.
hipError_t launch_decode(const void* K, int k_dtype, int64_t count, double scale, float* out, hipStream_t stream);

hipError_t launch_cost(const double* x, const double* y, int64_t n, int64_t m, int64_t d, int kind,
                       int normalize, double* C, int64_t ldc, double* blockmax, hipStream_t stream);
int64_t cost_blocks(int64_t n, int64_t m);

hipError_t launch_kernel_build(const double* C, int64_t ldc, int64_t n, int64_t m, double eps,
                               const double* f, const double* g, int k_dtype, void* K, int64_t ldk,
                               double store_scale, hipStream_t stream);

}  // namespace uot
