/*
 * uot.h -- C-ABI of the MI355X (gfx950) entropic unbalanced-OT Sinkhorn
 * library (libuot.so).
 *
 * The method (paper Section 2.1, with the four-part split of Section 4):
 * a non-negative n x m matrix is rescaled alternately by rows and by
 * columns, the factor of row i being (row target_i / row sum_i)^fi with
 * fi = tau/(tau+eps).  Written on scaling vectors, with the Gibbs kernel
 * K = exp(-C/eps) and the plan P = diag(u) K diag(v), one iteration is
 *
 *     row half-step     s = K v,      u = (a / s)^fi       (parts 4, 1)
 *     column half-step  w = K^T u,    v = (b / w)^fi       (parts 2, 3)
 *
 * rows first, from v = 1.  The library streams K once per iteration
 * (fused single pass; the paper's interleaving idea of Section 4.1 applied
 * to a read-only K) or twice (plain two-pass form, for comparison).
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer owned by the caller; the
 *    library never frees or retains it after the call returns.  Scratch
 *    memory comes only from the caller's workspace (ws, ws_bytes); the
 *    library allocates no device memory.  (It allocates one small pinned
 *    host buffer per process, once, to read the convergence flag.)
 *  - Matrices are row-major with a leading dimension (elements between the
 *    starts of consecutive rows).  Matrix base pointers must be 16-byte
 *    aligned and the leading dimension a multiple of 16/sizeof(element);
 *    otherwise UOT_ERR_ALIGN.  Vector pointers must be 8-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued on it; calls return before the GPU finishes unless stated.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and returned as a uot_status; uot_last_error() then describes them.
 *    Numerical trouble found on the GPU (non-finite scalings, a zero row or
 *    column sum with positive mass) is reported in uot_info.flags, which is
 *    device memory: read it after synchronising the stream.
 */
#ifndef UOT_H
#define UOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum uot_status {
    UOT_OK = 0,
    UOT_ERR_ARG = 1,          /* bad size, NULL pointer, eps <= 0, tau <= 0, ... */
    UOT_ERR_DTYPE = 2,        /* dtype not supported by this entry point */
    UOT_ERR_ALIGN = 3,        /* base or leading dimension not aligned */
    UOT_ERR_WORKSPACE = 4,    /* ws_bytes smaller than the size query returns */
    UOT_ERR_UNSUPPORTED = 5,  /* valid request outside the implemented envelope */
    UOT_ERR_HIP = 6           /* a HIP runtime call failed */
} uot_status;

typedef enum uot_dtype {
    UOT_F64 = 0,
    UOT_F32 = 1,
    UOT_BF16 = 2,             /* bfloat16, round-to-nearest-even from FP64 */
    UOT_FP8_E4M3 = 3          /* OCP E4M3FN (max 448), RNE with saturation */
} uot_dtype;

typedef enum uot_cost_kind {
    UOT_COST_SQEUCLID = 0,    /* C_ij = ||x_i - y_j||^2 */
    UOT_COST_COSINE = 1       /* C_ij = 1 - x_i . y_j  */
} uot_cost_kind;

typedef enum uot_accum {
    UOT_ACC_F32 = 0,          /* per-lane products and column partials in FP32 */
    UOT_ACC_F64 = 1           /* ... in FP64 (FP32 K only; FP64 K always uses FP64) */
} uot_accum;

/* uot_info.flags bits */
#define UOT_FLAG_NONFINITE     1u   /* a scaling became inf or NaN */
#define UOT_FLAG_ZERO_SUM      2u   /* a row or column sum was 0 with positive mass */
#define UOT_FLAG_NOT_CONVERGED 8u   /* tol > 0 and max_iter reached first */
#define UOT_FLAG_BARRIER_TIMEOUT 16u /* persistent loop: a grid-barrier wait hit its bound (results invalid) */

/* Device-resident solver report. */
typedef struct uot_info {
    int64_t iters;            /* iterations run */
    double err;               /* relative L1 change of the column marginal at the last iteration */
    int32_t absorptions;      /* log-domain absorptions performed */
    uint32_t flags;           /* UOT_FLAG_* */
} uot_info;

/* One UOT problem (Section 2.1).  a: n row targets, b: m column targets
 * (FP64, >= 0; a zero entry gives a zero scaling).  The kernel is given
 * either as K (k_dtype, K, ldk) or, when K is NULL, built from the FP64 cost
 * C (ldc) into the workspace in k_dtype.  eps > 0; tau > 0 or +inf
 * (balanced limit, fi = 1). */
typedef struct uot_problem {
    int64_t n, m;
    const double* a;
    const double* b;
    int32_t k_dtype;          /* uot_dtype of K */
    const void* K;            /* n x ldk, or NULL */
    int64_t ldk;
    const double* C;          /* n x ldc FP64 cost, or NULL (needed when K is NULL) */
    int64_t ldc;
    double eps;
    double tau;
    double k_scale;           /* given K only: the kernel is k_scale * K (0 = 1); use 1/448 for an
                                 FP8 K from uot_kernel_from_cost */
} uot_problem;

typedef struct uot_options {
    int32_t max_iter;         /* >= 0 iterations */
    int32_t check_every;      /* with tol > 0: host reads the stop flag every this many iterations (<= 0: 1) */
    double tol;               /* > 0: stop when the error is <= tol; <= 0: run exactly max_iter */
    int32_t fused;            /* 1: single pass over K per iteration; 0: plain row pass + column pass */
    int32_t accum;            /* uot_accum */
    double absorb_log_threshold;  /* > 0: log-domain absorption (needs C; see uot_sinkhorn); 0: off */
    int32_t checkpoint_every; /* k > 0: write v and K^T u every k iterations to outputs.ckpt
                                 (needs tol <= 0 and persistent = 0); 0 = none */
    int32_t tune;             /* 0: default launch shape; k > 0: use tuned shape index k-1 */
    const double* u0;         /* optional warm start (device, n), else u = 1 */
    const double* v0;         /* optional warm start (device, m), else v = 1 */
    int32_t persistent;       /* fused only: 1 = the whole loop in one cooperative launch with grid
                                 barriers (UOT_ERR_UNSUPPORTED when the grid cannot be co-resident
                                 or m > workgroup size * grid); 0 = two launches per iteration */
    int32_t store_iterates;   /* 1: write every iterate to outputs.ckpt (the reverse pass then reads
                                 them instead of re-running forward passes); needs checkpoint_every = 0,
                                 tol <= 0, persistent = 0 and no absorption; 0 = off */
} uot_options;

typedef struct uot_outputs {
    double* u;                /* required: device n, final u_T (FP64) */
    double* v;                /* required: device m, final v_T (FP64) */
    double* r;                /* optional: device n, row marginal u * (K v) */
    double* c;                /* optional: device m, column marginal v * (K^T u) */
    double* loss;             /* optional: device scalar, UOT objective of P_T */
    uot_info* info;           /* optional: device report */
    double* ckpt;             /* with options.checkpoint_every = k > 0: device buffer of
                                 (ceil(max_iter/k) + 1) x 2m doubles; slot c holds v and K^T u
                                 after iteration c*k (slot 0: the starting v).
                                 With options.store_iterates = 1 and T = max_iter: device buffer of
                                 (2T + 1) m + 2T n doubles, in four blocks: v_0 .. v_T (m each),
                                 K^T u_1 .. K^T u_T (m each), u_1 .. u_T (n each) and the row sums
                                 K v_0 .. K v_{T-1} (n each) */
    double* f;                /* optional: device n, eps * log(u_T) (finite where u_T overflows) */
    double* g;                /* optional: device m, eps * log(v_T) */
} uot_outputs;

/* Per-kernel durations of one uot_sinkhorn_profiled call, measured with HIP
 * events recorded on `stream` around every launch of every 8th iteration
 * (counts below are those timed launches), plus the whole loop. */
typedef struct uot_profile {
    int32_t fused_launches;   /* timed single-pass launches (row + column half-steps) */
    float fused_ms;           /* their summed duration */
    int32_t row_launches;     /* plain row-pass launches */
    float row_ms;
    int32_t col_launches;     /* plain column-pass launches */
    float col_ms;
    int32_t finalize_launches;
    float finalize_ms;
    float loop_ms;            /* whole iteration loop (all iterations) */
} uot_profile;

/* Tail of a packed batch descriptor block (host memory; see uot_batched_pack). */
typedef struct uot_batched_meta {
    int32_t count;            /* problems in the block */
    int32_t k_dtype;          /* their common K dtype */
    int64_t m_lds;            /* FP64 values per LDS vector the launch needs */
    int32_t items;            /* queue entries (a split problem has one per part) */
    int32_t nsplit;           /* problems split over several workgroups */
    int64_t pool_bytes;       /* workspace bytes their exchanges use */
} uot_batched_meta;

/* Status text, and a thread-local description of the last error. */
const char* uot_status_string(uot_status s);
const char* uot_last_error(void);

/*
 * Dense FP64 cost from points (the cost C whose Gibbs kernel is rescaled,
 * Section 2.1).  x: n x d, y: m x d (FP64, row-major, contiguous).
 * kind: uot_cost_kind.  normalize_max != 0 divides the whole matrix by its
 * maximum (when that maximum is > 0).  C: n x ldc FP64 output, ldc >= m.
 * Workspace: uot_cost_workspace_size(n, m) bytes (for the max reduction).
 * Errors: UOT_ERR_ARG for n, m, d <= 0 or NULL pointers; UOT_ERR_WORKSPACE.
 */
size_t uot_cost_workspace_size(int64_t n, int64_t m);
uot_status uot_cost_from_points(const double* x, const double* y, int64_t n, int64_t m,
                                int64_t d, int32_t kind, int32_t normalize_max,
                                double* C, int64_t ldc, void* ws, size_t ws_bytes,
                                void* stream);

/*
 * Gibbs kernel K_ij = exp((f_i + g_j - C_ij)/eps) (Section 2.1's matrix A,
 * built from its cost), evaluated in FP64 and rounded to nearest-even into
 * k_dtype (F64, F32, BF16; FP8 stores RNE(448 K) saturated at 448, so pass
 * k_scale = 1/448 with it).  f, g: optional FP64 potentials (NULL = 0).
 * C: n x ldc FP64.  K: n x ldk output; padding columns [m, ldk) are 0.
 * BF16 values below 2^-126 are stored as 0; FP8 keeps its subnormals
 * (multiples of 2^-9), so only 448 K below 2^-10 becomes 0.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN.
 */
uot_status uot_kernel_from_cost(const double* C, int64_t ldc, int64_t n, int64_t m,
                                double eps, const double* f, const double* g,
                                int32_t k_dtype, void* K, int64_t ldk, void* stream);

/*
 * Workspace bytes that uot_sinkhorn needs for this problem and options
 * (0 on invalid arguments).
 */
size_t uot_sinkhorn_workspace_size(const uot_problem* prob, const uot_options* opt);

/*
 * The UOT Sinkhorn scaling loop (Section 2.1; Section 4's interleaved
 * single pass when opt->fused != 0).  Runs up to opt->max_iter iterations
 * of the row then column half-step from v = 1 (or the warm start), stops
 * early when tol > 0 and the relative L1 change of the column marginal
 * c = v * (K^T u) is <= tol, then forms the marginals and the objective
 *     <C,P> + eps sum P(log P - 1) + tau KL~(P1|a) + tau KL~(P^T1|b)
 * (KL~(x|y) = sum x log(x/y) - x + y; the KL terms are dropped for
 * tau = inf) in FP64 from O(n+m) quantities.
 *
 * K dtypes: UOT_F64, UOT_F32, UOT_BF16, UOT_FP8_E4M3 (BF16 and FP8: fused,
 * FP32 lane arithmetic).  Scalings and all reductions across lanes and
 * workgroups are FP64 (opt->accum picks the per-lane type for FP32 K).
 * Results are bitwise reproducible for a fixed problem and launch shape.
 * With tol > 0 the host synchronises on `stream` every check_every
 * iterations; with tol <= 0 the call only enqueues work.
 *
 * Log-domain absorption (opt->absorb_log_threshold > 0; needs C): the state
 * is (f, g, u, v) with totals u e^{f/eps}, v e^{g/eps}, and the stored
 * kernel is Kt_ij = exp((f_i + g_j - C_ij)/eps).  Whenever Kt is built, f
 * and g are normalised, f_i = min_j (C_ij - g_j) and then
 * g_j = min_i (C_ij - f_i), so every row's and every column's largest entry
 * is exactly 1 (u, v are rescaled to keep the totals).  The updates become
 *     u = (a / (Kt v))^fi e^{-(1-fi) f/eps},  v = (b / (Kt^T u))^fi e^{-(1-fi) g/eps},
 * the same iterates in exact arithmetic.  Every check_every iterations, if
 * max |log u| or max |log v| exceeds the threshold, v is absorbed (g += eps
 * log v, v = 1), f, g are normalised again and Kt is rebuilt from C.  Kt
 * lives in the workspace in k_dtype (FP8: 448 Kt).  outputs->u, v then receive
 * the totals (inf where they overflow FP64) and outputs->f, g the finite
 * potentials eps log(total); info->absorptions counts the absorptions.
 *
 * Errors: UOT_ERR_ARG (n or m < 1, NULL a/b/u/v, eps <= 0, tau <= 0,
 * max_iter < 0, neither K nor C, absorption without C), UOT_ERR_DTYPE,
 * UOT_ERR_ALIGN, UOT_ERR_WORKSPACE, UOT_ERR_UNSUPPORTED (m above the row
 * length one workgroup holds: 16384 FP32, 8192 FP64, 32768 BF16, 65536 FP8;
 * combinations outside the envelope stated at each option), UOT_ERR_HIP.
 */
uot_status uot_sinkhorn(const uot_problem* prob, const uot_options* opt,
                        const uot_outputs* out, void* ws, size_t ws_bytes, void* stream);

/*
 * The paper's literal form (Section 2.1, in the single-pass order of
 * Section 4.1's Algorithm 1): the matrix given as prob->K (FP32 or FP64,
 * n x ldk) is rescaled IN PLACE.  Before the first iteration the column
 * factors beta_j = (b_j / column sum_j)^fi are formed; each iteration then
 * multiplies every row by beta, forms the row factor alpha_i =
 * (a_i / row sum_i)^fi, multiplies the row by it (one read and one write of
 * the matrix, fused), and forms the next beta from the new column sums.
 * For fi = 1 (tau = inf) this is the vector-form iteration taken columns
 * first; for fi < 1 it is a different iteration (its limit does not depend
 * on the cost), provided to measure the in-place form beside the vector
 * form (twice the bytes per iteration).
 *   prob: n, m, a, b (targets), K (the matrix, modified), ldk, eps, tau;
 *     k_scale 0 or 1; C ignored.
 *   opt: max_iter, tol / check_every (relative L1 change of beta * column
 *     sums, as uot_sinkhorn), tune (one-row launch shapes 1-8); absorption,
 *     checkpoints, warm start, cooperative loop and FP64 accumulation of an
 *     FP32 matrix must be off.
 *   out: u (n) receives the last row factors, v (m) the column factors the
 *     next iteration would apply, r (n, optional) the row sums and c (m,
 *     optional) the column sums of the rescaled matrix, info (optional);
 *     loss, ckpt, f, g are ignored.
 * Columns [m, round up of m to 16 bytes) of each row are written as 0.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE,
 * UOT_ERR_UNSUPPORTED, UOT_ERR_HIP.
 */
size_t uot_matrix_rescale_workspace_size(const uot_problem* prob, const uot_options* opt);
uot_status uot_matrix_rescale(const uot_problem* prob, const uot_options* opt, const uot_outputs* out,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel-free solve for a squared-Euclidean cost of points (Section 2.1's
 * iteration in vector form, as uot_sinkhorn with opt->fused = 1): the
 * Gibbs kernel K_ij = exp(-cost_scale ||x_i - y_j||^2 / eps) is recomputed
 * inside every pass instead of being read from memory, so no n x m array
 * exists and the per-iteration memory traffic is O(n + m) (the O(nm)
 * traffic Sections 1 and 3 name as the bottleneck is gone; the pass is
 * bounded by the vector ALU instead).  Each entry is formed from
 * t = -cost_scale log2(e) ||x_i - y_j||^2 / eps, evaluated in FP64 as
 * alpha_i + beta_j + x'_i . y_j, as 2^t = 2^rint(t) 2^(t - rint(t)), the
 * fractional power by the hardware exp2 on its FP32 rounding (relative
 * error about 1e-7 per entry, the size of an FP32 storage rounding of K);
 * the products with v and u and the column partials are FP32 per lane,
 * every reduction across lanes and workgroups FP64, as for an FP32 K.
 *   prob: n, m, a, b, eps, tau (K, C, ldk, ldc, k_dtype, k_scale ignored)
 *   x, y, dim   source points (n x dim) and target points (m x dim), FP64
 *               row-major, contiguous, dim 2 or 3
 *   cost_scale  > 0; the cost is cost_scale ||x_i - y_j||^2 (pass
 *               1 / max_ij ||x_i - y_j||^2 to match a max-normalised cost)
 *   opt: max_iter, tol, check_every, u0, v0 as uot_sinkhorn; fused = 1,
 *     accum = UOT_ACC_F32, and no absorption, checkpoints or cooperative
 *     loop (else UOT_ERR_UNSUPPORTED)
 *   out: as uot_sinkhorn (u, v required; r, c, loss, info, f, g optional;
 *     ckpt ignored)
 * Rows of up to 8192 columns run one fused pass per iteration (a workgroup
 * keeps the target points of a whole row on chip); wider rows (m up to
 * 2^20, else UOT_ERR_UNSUPPORTED) run in column tiles of 8192: a row pass
 * (each tile's row sums), the row scalings, then a column pass, each pass
 * forming K again, so an iteration costs twice the arithmetic of the fused
 * pass.  The workspace then also holds ceil(m / 8192) doubles per row.
 * Errors: UOT_ERR_ARG, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE, UOT_ERR_UNSUPPORTED,
 * UOT_ERR_HIP.  Workspace: uot_sinkhorn_points_workspace_size bytes (0 on
 * invalid arguments).
 */
size_t uot_sinkhorn_points_workspace_size(const uot_problem* prob, int64_t dim, double cost_scale,
                                          const uot_options* opt);
uot_status uot_sinkhorn_points(const uot_problem* prob, const double* x, const double* y, int64_t dim,
                               double cost_scale, const uot_options* opt, const uot_outputs* out,
                               void* ws, size_t ws_bytes, void* stream);

/* Decreasing-eps schedule of uot_sinkhorn_lse (host memory). */
typedef struct uot_eps_schedule {
    double eps0;              /* first stage's eps; <= prob->eps: no schedule */
    double factor;            /* eps_{k+1} = max(eps, eps_k * factor), 0 < factor < 1 */
    int32_t stage_iters;      /* iterations of every stage before the one at eps (>= 1) */
    int32_t reserved;
} uot_eps_schedule;

/*
 * Log-domain (log-sum-exp) solve: the iteration of Section 2.1 (vector
 * form, rows first) carried on the potentials f = eps log u, g = eps log v,
 *     f_i = fi (eps log a_i - eps LSE_j((g_j - C_ij)/eps))
 *     g_j = fi (eps log b_j - eps LSE_i((f_i - C_ij)/eps)),
 * every sum taken under its maximum, so no exponential exceeds 1 at any
 * eps: no absorption is needed where the scalings leave the FP64 range.
 * One fused pass per iteration reads the cost C once; the exponents are
 * formed in FP64 and each exponential is the hardware exp2 (FP32, relative
 * error about 1e-7 on the terms that carry the sums), summed in FP32 per
 * lane and in FP64 across lanes and workgroups.
 *   prob: n, m, a, b, C (FP64, n x ldc, 16-byte aligned, even ldc >= m),
 *     eps, tau; k_dtype chooses the cost the passes read: UOT_F64 (C
 *     itself, 8 bytes per entry and iteration) or UOT_F32 (C rounded to
 *     FP32 once into the workspace, 4 bytes; its rounding moves each
 *     exponent by up to |C_ij|/eps * 2^-24, so it suits costs with
 *     |C|/eps well below 2^24 * 1e-6).  K, ldk, k_scale ignored.
 *   sched: NULL, or a schedule: stages at eps0, eps0 factor, ... down to
 *     eps, each before the last running stage_iters iterations from the
 *     previous stage's potentials; the stage at eps runs up to max_iter
 *     iterations with the stopping rule of uot_sinkhorn (its first
 *     iteration is compared with a zero marginal).
 *   opt: max_iter, tol, check_every; fused = 1, accum = UOT_ACC_F32 and no
 *     absorption, checkpoints, cooperative loop or warm start (else
 *     UOT_ERR_UNSUPPORTED).
 *   out: u, v (required) receive the totals e^{f/eps}, e^{g/eps} (inf where
 *     they leave the FP64 range), f, g (optional) the potentials, r, c,
 *     loss, info as uot_sinkhorn (info.iters counts every stage's iterations).
 * Rows of at most 8192 columns.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE,
 * UOT_ERR_UNSUPPORTED, UOT_ERR_HIP.  Workspace:
 * uot_sinkhorn_lse_workspace_size bytes (0 on invalid arguments).
 */
size_t uot_sinkhorn_lse_workspace_size(const uot_problem* prob, const uot_options* opt,
                                       const uot_eps_schedule* sched);
uot_status uot_sinkhorn_lse(const uot_problem* prob, const uot_options* opt, const uot_eps_schedule* sched,
                            const uot_outputs* out, void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): uot_sinkhorn without a
 * workspace argument.  Its scratch is a device array of the library,
 * UOT_NOALLOC_SCRATCH_BYTES (64 MiB), one copy per GPU held until the
 * process ends; the call makes no hipMalloc, hipFree or other allocation
 * and never waits on `stream`.
 *   - Same problem, options and outputs as uot_sinkhorn, same kernels and
 *     results (bit for bit), on the current device (hipGetDevice); `stream`
 *     must belong to it.
 *   - The problem's workspace (uot_sinkhorn_workspace_size) must be at most
 *     UOT_NOALLOC_SCRATCH_BYTES, else UOT_ERR_WORKSPACE (e.g. a 16384^2 FP32
 *     K with FP32 accumulation needs about 17 MiB; a K built inside the
 *     call from C needs n x ldk more and rarely fits).
 *   - With tol > 0 all max_iter iterations are enqueued; the launches after
 *     the stopping test passed return at once (info.iters as uot_sinkhorn).
 *   - Absorption (opt->absorb_log_threshold > 0) is refused with
 *     UOT_ERR_UNSUPPORTED: it decides on the host.
 *   - Every call on one GPU uses that GPU's scratch, which keeps the last
 *     call's contents (each call re-initialises what it reads first): calls
 *     that overlap on one GPU (two streams, two host threads) race and must
 *     be ordered by the caller.
 * Errors: as uot_sinkhorn, plus UOT_ERR_WORKSPACE (above the scratch size),
 * UOT_ERR_UNSUPPORTED (absorption; device index above 63), UOT_ERR_HIP.
 */
#define UOT_NOALLOC_SCRATCH_BYTES (64ull << 20)
uot_status uot_sinkhorn_noalloc(const uot_problem* prob, const uot_options* opt,
                                const uot_outputs* out, void* stream);

/* uot_sinkhorn with HIP-event timing of the streaming kernels written to
 * *prof (host pointer).  Synchronises `stream` before returning. */
uot_status uot_sinkhorn_profiled(const uot_problem* prob, const uot_options* opt,
                                 const uot_outputs* out, void* ws, size_t ws_bytes,
                                 void* stream, uot_profile* prof);

/*
 * Gradient of the objective returned by uot_sinkhorn (the loop unrolled
 * for exactly opt->max_iter iterations from v = 1, differentiated in
 * reverse mode; the paper gives no gradient, this is the exact derivative of
 * the iteration of Section 2.1 as written above).  Each reverse step streams
 * K once: row dots with the adjoint column vector (and, for point gradients,
 * with it and v_{t-1} times each coordinate of y), then the column partials
 * of K^T sbar.  Iterates are recomputed segment by segment from the
 * checkpoints of the forward call (same problem and options, including
 * checkpoint_every; the forward must not have been given u0/v0), or, when
 * the forward stored every iterate (options.store_iterates = 1), read from
 * that record with no forward pass repeated (one pass over K per reverse
 * step instead of two; the gradients are the same to the bit, since the
 * recomputed iterates are).
 *
 * The adjoint of K, Kbar, is a sum of 2T + 2 rank-1 terms (two per
 * iteration, two from the objective); dL/dC_ij = -Kbar_ij K_ij / eps.  When
 * grad_C or grad_y is requested the reverse passes store the terms' factors
 * in the workspace ((2T + 2) (n + m) doubles) and one FP64 matrix product
 * on the matrix cores with inner dimension 2T + 2 forms dL/dC, K applied in
 * its epilogue.
 *
 *   u, v        forward results u_T, v_T (device, n and m)
 *   ckpt        the forward's outputs.ckpt (checkpoints or the stored iterates)
 *   grad_loss   device scalar g; outputs are g times dL/d(input)
 *   grad_a      device n or NULL;  grad_b  device m or NULL
 *   grad_C      device n x ldgc FP64 (row-major, ldgc >= m; columns [m, ldgc)
 *               untouched) or NULL: g dL/dC, with C the cost that built K
 *               (K = exp(-C/eps), the stored K used in the product)
 *   x, y, dim   source (n x dim) and target (m x dim) points, row-major FP64,
 *               of a squared-Euclidean cost C_ij = ||x_i - y_j||^2 that was
 *               not max-normalised; dim 0 (no point gradient), 2 or 3
 *   grad_x      device n x dim or NULL: dL/dx_i = 2 sum_j G_ij (x_i - y_j),
 *               G = dL/dC, from row sums formed inside the reverse passes
 *   grad_y      device m x dim or NULL: dL/dy_j = 2 sum_i G_ij (y_j - x_i),
 *               from column sums in the product's epilogue (needs x)
 *
 * Requirements: max_iter >= 1, checkpoint_every >= 1 or store_iterates = 1
 * (not both), tol <= 0, histogram
 * entries > 0, rows of at most 8192 columns (FP32 or FP64 K).
 * Errors: UOT_ERR_ARG, UOT_ERR_UNSUPPORTED, UOT_ERR_WORKSPACE, UOT_ERR_ALIGN,
 * UOT_ERR_HIP.  Workspace: uot_sinkhorn_backward_workspace_size bytes, with
 * cost_grad != 0 when grad_C or grad_y will be requested.
 */
size_t uot_sinkhorn_backward_workspace_size(const uot_problem* prob, const uot_options* opt, int64_t dim,
                                            int32_t cost_grad);
uot_status uot_sinkhorn_backward(const uot_problem* prob, const uot_options* opt,
                                 const double* u, const double* v, const double* ckpt,
                                 const double* grad_loss, double* grad_a, double* grad_b,
                                 double* grad_C, int64_t ldgc,
                                 const double* x, const double* y, int64_t dim,
                                 double* grad_x, double* grad_y,
                                 void* ws, size_t ws_bytes, void* stream);

/*
 * Implicit (envelope) gradient of the objective at the scalings (u, v) of a
 * converged uot_sinkhorn call: at the minimiser P of the objective its
 * derivative in a parameter is the partial derivative at fixed P, so
 *   dL/dC = P = diag(u) K diag(v),  dL/da = tau (1 - r/a),  dL/db = tau (1 - c/b),
 *   dL/dx_i = 2 sum_j P_ij (x_i - y_j),  dL/dy_j = 2 sum_i P_ij (y_j - x_i)
 * (r = P 1, c = P^T 1; the KL terms vanish for tau = inf).  This equals the
 * gradient of the unrolled loop only as far as (u, v) has converged (the
 * difference shrinks like fi^(2T)); it costs one marginal pass over K (r and
 * c), plus one per point coordinate when x or y gradients are requested
 * (K (v y_d) by rows and K^T (u x_d) by columns in the same pass), plus the
 * dense write of dL/dC if requested -- instead of the 3T passes of the
 * unrolled reverse sweep.  No checkpoints are needed.
 *
 *   prob, opt   the forward's problem (K of any dtype, or C to rebuild it)
 *               and options (accum, tune; the loop options are ignored)
 *   u, v        the forward's scalings (device, n and m; finite: not the
 *               totals of an absorbed solve)
 *   grad_loss   device scalar g; outputs are g times dL/d(input)
 *   grad_a, grad_b        device n, m or NULL
 *   grad_C      device n x ldgc FP64 or NULL (columns [m, ldgc) untouched)
 *   x, y, dim   points of an un-normalised squared-Euclidean cost (dim 1..16)
 *   grad_x, grad_y        device n x dim, m x dim or NULL
 * Requirements: a, b > 0 where gradients are requested.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE,
 * UOT_ERR_UNSUPPORTED, UOT_ERR_HIP.  Workspace:
 * uot_sinkhorn_implicit_backward_workspace_size bytes.
 */
size_t uot_sinkhorn_implicit_backward_workspace_size(const uot_problem* prob, const uot_options* opt, int64_t dim);
uot_status uot_sinkhorn_implicit_backward(const uot_problem* prob, const uot_options* opt,
                                          const double* u, const double* v, const double* grad_loss,
                                          double* grad_a, double* grad_b, double* grad_C, int64_t ldgc,
                                          const double* x, const double* y, int64_t dim,
                                          double* grad_x, double* grad_y,
                                          void* ws, size_t ws_bytes, void* stream);

/*
 * Decode `count` stored kernel entries (a multiple of 16 bytes' worth) to
 * FP32 exactly as the streaming passes read them, times k_scale.  For
 * inspecting a stored K (e.g. checking the FP8 decoding).
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_HIP.
 */
uot_status uot_kernel_to_f32(const void* K, int32_t k_dtype, int64_t count, double k_scale, float* out,
                             void* stream);

/*
 * The plan P = diag(u) K diag(v) of Section 2.1's rescaled matrix, written
 * densely on request (n x ldp, row-major, FP64 or FP32; columns [m, ldp)
 * untouched).  Two forms:
 *  - prob->K with u, v (e.g. outputs->u, v of uot_sinkhorn):
 *      P_ij = u_i (k_scale K_ij) v_j, products in FP64;
 *  - prob->C with f, g (outputs->f, g: potentials of the total scalings,
 *    finite where u, v overflow, as after absorption):
 *      P_ij = exp((f_i + g_j - C_ij) / prob->eps), in FP64.
 * K is used when prob->K, u and v are all given, else C with f and g.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_HIP.
 */
uot_status uot_plan(const uot_problem* prob, const double* u, const double* v, const double* f, const double* g,
                    void* plan, int64_t ldp, int32_t plan_dtype, void* stream);

/*
 * R histogram pairs sharing one kernel (each pair an independent instance
 * of Section 2.1's loop): the two half-steps of an iteration become two
 * matrix products on the matrix cores,
 *     S = K V,    U = (A / S)^fi,      W = K^T U,   V = (B / W)^fi,
 * with V = 1 at the start, then r = U (K V), c = V (K^T U) and the
 * objective of every pair (as uot_sinkhorn) in FP64.
 * shared: n, m, K (UOT_F32 or UOT_BF16; padding columns [m, ldk) finite),
 *   ldk, k_scale, eps, tau; a, b and C are ignored.
 * A: R x n and B: R x m FP64, histogram r in row r (A[r*n + i] = a_r,i).
 * U: R x n, V: R x m FP64 outputs (same layout); losses: R FP64;
 * info: one record for all pairs (iters, flags).
 * Arithmetic: BF16 K with each right-hand side split into a bfloat16 high
 * part and the bfloat16 rounding of the remainder (two products per tile,
 * ~16 significant bits of the right-hand side kept); FP32 K with FP32
 * products.  Each reduction is split over k into chunks summed in FP32 on
 * the matrix cores and added in FP64 in a fixed order.
 * opt: max_iter >= 1 iterations exactly; tol, absorption, checkpoints, warm
 * start and the cooperative loop must be off (else UOT_ERR_UNSUPPORTED);
 * tune selects the product kernel of the BF16 form (the FP32 form always
 * stages 128 x 128 tiles through LDS): 0 (default) or 3, 256 x 256 tiles
 * over tiled copies of K and K^T when R is a multiple of 256 (else as 1);
 * 1, 128 x 128 tiles staged through LDS; 2, each wave loads its own
 * operand fragments; 4, 128 x 128 tiles over the tiled copies.  Other
 * values: UOT_ERR_ARG.  The tiled copies take the workspace of a second K.
 * Workspace (uot_sinkhorn_multi_workspace_size): a transposed copy of K
 * (or, for the tiled BF16 products, tiled copies of K and K^T), the split
 * partial sums and the right-hand-side planes.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE,
 * UOT_ERR_UNSUPPORTED, UOT_ERR_HIP.
 */
size_t uot_sinkhorn_multi_workspace_size(const uot_problem* shared, int32_t R, const uot_options* opt);
uot_status uot_sinkhorn_multi(const uot_problem* shared, int32_t R, const double* A, const double* B,
                              const uot_options* opt, double* U, double* V, double* losses, uot_info* info,
                              void* ws, size_t ws_bytes, void* stream);


/*
 * Many independent problems of uneven size, solved in ONE persistent launch
 * (each problem is an independent application of the loop of Section 2.1;
 * the single-pass interleave of Section 4.1 is applied inside one
 * workgroup per problem).
 *
 * Each workgroup takes problems from a device queue in longest-first order
 * (estimated time: the rows each row group of the problem's tile shape steps
 * through, weighted by the chunks per lane) and runs all of a problem's
 * iterations by itself; no grid-wide synchronisation, no host round trip.
 * A problem whose estimated time exceeds the average per resident
 * workgroup is split by rows into up to 4 queue entries that run side by
 * side on as many workgroups and exchange their column sums once per
 * iteration (at most 256 split problems, whose parts take at most 3/4 of
 * the resident workgroups; split problems are queued first, so all parts
 * of a problem run at the same time).  Products, row sums and column sums are FP64 on
 * the widened stored K; a split problem adds its parts' column sums in part
 * order, so its result is the same FP64 iteration up to summation order.
 * Every problem
 * runs exactly opt->max_iter iterations, or stops after the first check
 * (every check_every iterations) whose relative L1 change of the column
 * marginal is <= opt->tol, then forms r = u*(K v), c = v*(K^T u) and the
 * objective (as uot_sinkhorn) into its outputs.
 *
 * probs[i]: K (required; all problems share one k_dtype; n*ldk*sizeof(K)
 *   below 2 GiB; m at most 2048 for FP64/FP32/BF16 and 4096 for FP8),
 *   a, b, eps, tau, k_scale.  C is ignored.
 * outs[i]: u, v, r, c (FP64 device vectors), loss, info (required); ckpt,
 *   f, g ignored.
 * opt: max_iter, tol, check_every, tune (> 0: time the candidate tile
 *   shapes of each column-count bucket first, see uot_batched_tune); the
 *   absorption, checkpoint, warm-start and cooperative options must be off
 *   (else UOT_ERR_UNSUPPORTED).
 * Workspace: uot_sinkhorn_batched_workspace_size(count) bytes, 256-byte
 * aligned (queue head, descriptors, exchange pool of the split problems).
 * This call copies the descriptors from pageable host memory and
 * synchronises `stream` once before launching; use the packed form below
 * to capture the launch in a HIP graph.
 * Errors: UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE,
 * UOT_ERR_UNSUPPORTED, UOT_ERR_HIP.
 */
size_t uot_sinkhorn_batched_workspace_size(int32_t count);
uot_status uot_sinkhorn_batched(const uot_problem* probs, int32_t count, const uot_options* opt,
                                const uot_outputs* outs, void* ws, size_t ws_bytes, void* stream);

/*
 * Two-step form of uot_sinkhorn_batched whose launch step makes no host
 * synchronisation and no host-to-device copy, so that it can be captured
 * in a HIP graph and replayed.
 * uot_batched_pack (host only) validates the problems and writes the
 * descriptor block into desc_host (uot_batched_desc_bytes(count) bytes):
 * first the device descriptors (copy those uot_batched_desc_bytes(count) -
 * sizeof(uot_batched_meta) bytes to 16-byte aligned device memory), then a
 * uot_batched_meta.  The descriptors hold the problems' device pointers:
 * they must stay valid while the block is used.
 * meta->items queue entries are written (count plus one more per extra part
 * of a split problem; the index word of each descriptor names its problem).
 * Splitting needs the device's resident workgroup count, so a pack without
 * a device splits nothing.
 * uot_sinkhorn_batched_packed enqueues the reset of the queue and of the
 * split problems' counters, and the persistent launch; ws as for
 * uot_sinkhorn_batched.  trace (optional, device, 2*meta->items uint64): per
 * queue entry the device wall clock when a workgroup took it and when it
 * finished; uot_device_wall_clock_khz gives the clock's rate.
 * uot_batched_tune runs only the autotuning step (results are kept for the
 * process, per K dtype and column-count bucket, and used by later packs).
 */
size_t uot_batched_desc_bytes(int32_t count);
uot_status uot_batched_pack(const uot_problem* probs, int32_t count, const uot_options* opt,
                            const uot_outputs* outs, void* desc_host, size_t desc_bytes);
uot_status uot_sinkhorn_batched_packed(const void* desc_dev, const uot_batched_meta* meta,
                                       const uot_options* opt, void* ws, size_t ws_bytes,
                                       uint64_t* trace, void* stream);
uot_status uot_batched_tune(const uot_problem* probs, int32_t count, const uot_options* opt,
                            const uot_outputs* outs, void* ws, size_t ws_bytes, void* stream);
int64_t uot_device_wall_clock_khz(void);

#ifdef __cplusplus
}
#endif

#endif /* UOT_H */
