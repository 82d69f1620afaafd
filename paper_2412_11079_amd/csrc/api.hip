// C-ABI of libuot.so: argument checks, workspace layout, launch sequence.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "uot_common.h"

using namespace uot;

namespace {

thread_local std::string g_last_error;

uot_status fail(uot_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
uot_status fail(uot_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

uot_status hip_fail(hipError_t e, const char* what) {
    return fail(UOT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define UOT_HIP(call, what)                              \
    do {                                                 \
        hipError_t e__ = (call);                         \
        if (e__ != hipSuccess) return hip_fail(e__, what); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int elem_size(int dt) {
    switch (dt) {
        case UOT_F64: return 8;
        case UOT_F32: return 4;
        case UOT_BF16: return 2;
        case UOT_FP8_E4M3: return 1;
        default: return 0;
    }
}

// Pinned host word used to read the stop flag (allocated once per process).
std::once_flag g_pinned_once;
uint32_t* g_pinned = nullptr;
hipError_t g_pinned_err = hipSuccess;

uint32_t* pinned_flag() {
    std::call_once(g_pinned_once, [] {
        g_pinned_err = hipHostMalloc((void**)&g_pinned, 64, hipHostMallocDefault);
        if (g_pinned_err != hipSuccess) g_pinned = nullptr;
    });
    return g_pinned;
}

// Event pool for profiled runs (grown on demand, kept for the process).
std::mutex g_ev_mu;
std::vector<hipEvent_t> g_events;

hipError_t events(size_t count, std::vector<hipEvent_t>& out) {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    while (g_events.size() < count) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        g_events.push_back(e);
    }
    out.assign(g_events.begin(), g_events.begin() + count);
    return hipSuccess;
}

// Launch plan for one solve.
struct Plan {
    int k_dtype;
    int acc64;
    int vec;              // elements per 16-byte chunk of K
    int shape;            // index into the pass shape table
    int32_t G;            // row strips
    int64_t rows_per_wg;
    int64_t ldp;          // partial row stride (elements)
    int64_t ldk_ws;       // leading dimension of a K built into the workspace
    int64_t ldv_bytes;    // LDS bytes holding v (shapes with v in LDS)
    size_t lds_bytes;     // LDS per workgroup (estimate incl. static)
    bool persistent;      // whole loop in one cooperative launch
    int32_t fin_cols;     // persistent: columns finalized per workgroup
    int64_t scratch_bytes;  // persistent: LDS before the row strips
    int32_t fin_blocks;   // blocks that write stopping-test sums
    bool build_k;
    // workspace offsets
    size_t off_ctrl, off_cprev, off_w, off_s, off_bp, off_part, off_k, total;
};

uot_status check_problem(const uot_problem* p, const uot_options* o) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "empty problem (n=%lld, m=%lld)", (long long)p->n, (long long)p->m);
    if (!p->a || !p->b) return fail(UOT_ERR_ARG, "a and b must not be NULL");
    if (!aligned(p->a, 8) || !aligned(p->b, 8)) return fail(UOT_ERR_ALIGN, "a and b must be 8-byte aligned");
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "tau must be > 0 (or +inf)");
    if (o->max_iter < 0) return fail(UOT_ERR_ARG, "max_iter must be >= 0");
    if (o->absorb_log_threshold != 0.0)
        return fail(UOT_ERR_UNSUPPORTED, "log-domain absorption is not available in this entry point");
    if (o->checkpoint_every != 0) return fail(UOT_ERR_UNSUPPORTED, "checkpoints are not available in this entry point");
    if (p->k_dtype != UOT_F64 && p->k_dtype != UOT_F32)
        return fail(UOT_ERR_DTYPE, "K dtype %d not supported (FP64, FP32)", (int)p->k_dtype);
    const int es = elem_size(p->k_dtype);
    const int vec = 16 / es;
    if (p->K) {
        if (p->ldk < p->m) return fail(UOT_ERR_ARG, "ldk (%lld) < m (%lld)", (long long)p->ldk, (long long)p->m);
        if (!aligned(p->K, 16) || p->ldk % vec != 0)
            return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned with ldk a multiple of %d", vec);
    } else {
        if (!p->C) return fail(UOT_ERR_ARG, "either K or C must be given");
        if (p->ldc < p->m) return fail(UOT_ERR_ARG, "ldc (%lld) < m (%lld)", (long long)p->ldc, (long long)p->m);
        if (!aligned(p->C, 8)) return fail(UOT_ERR_ALIGN, "C must be 8-byte aligned");
    }
    if (o->u0 && !aligned(o->u0, 8)) return fail(UOT_ERR_ALIGN, "u0 must be 8-byte aligned");
    if (o->v0 && !aligned(o->v0, 8)) return fail(UOT_ERR_ALIGN, "v0 must be 8-byte aligned");
    return UOT_OK;
}

int default_shape(int64_t nv) {
    // Smallest instantiated shape whose lanes cover a row (in 16-byte chunks).
    static const int order[] = {0, 1, 2, 3, 4, 6};
    for (int idx : order) {
        PassShape s = pass_shape(idx);
        if ((int64_t)s.wg * s.nc >= nv) return idx;
    }
    return -1;
}

// Largest dynamic LDS one workgroup may use on the current device.
int64_t max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

uot_status make_plan(const uot_problem* p, const uot_options* o, Plan& P) {
    uot_status st = check_problem(p, o);
    if (st != UOT_OK) return st;
    P.k_dtype = p->k_dtype;
    P.acc64 = (p->k_dtype == UOT_F64) || (o->accum == UOT_ACC_F64);
    P.vec = 16 / elem_size(p->k_dtype);
    const int64_t nv = (p->m + P.vec - 1) / P.vec;
    if (o->tune > 0) {
        if (o->tune > pass_shape_count()) return fail(UOT_ERR_ARG, "tune index %d out of range", o->tune);
        P.shape = o->tune - 1;
        PassShape s = pass_shape(P.shape);
        if ((int64_t)s.wg * s.nc < nv)
            return fail(UOT_ERR_UNSUPPORTED, "shape %d covers %lld columns, m=%lld", P.shape,
                        (long long)s.wg * s.nc * P.vec, (long long)p->m);
    } else {
        P.shape = default_shape(nv);
        if (P.shape < 0)
            return fail(UOT_ERR_UNSUPPORTED, "m=%lld exceeds the row length one workgroup holds (%d columns)",
                        (long long)p->m, 4096 * P.vec);
    }
    PassShape s = pass_shape(P.shape);
    P.ldp = round_up(p->m, 64);
    P.ldv_bytes = round_up(round_up(p->m, P.vec) * (P.acc64 ? 8 : 4), 16);
    P.persistent = o->persistent != 0;
    if (P.persistent && !o->fused)
        return fail(UOT_ERR_ARG, "the persistent loop runs the fused pass only");
    int64_t target = 256LL * (1024 / s.wg);     // about one wave of workgroups on 256 CUs
    if (P.persistent) {
        // LDS: max(v, finalize scratch of 4 doubles per thread), then the row strips
        P.scratch_bytes = round_up(std::max<int64_t>(s.vlds ? P.ldv_bytes : 0, (int64_t)s.wg * 32), 16);
        int64_t rows_guess = (p->n + 255) / 256;
        size_t lds_guess = (size_t)P.scratch_bytes + 2 * sizeof(double) * (size_t)rows_guess;
        int gmax = persist_max_grid(P.k_dtype, P.acc64, P.shape, lds_guess);
        if (gmax <= 0) return fail(UOT_ERR_UNSUPPORTED, "shape %d cannot run as a cooperative launch", P.shape);
        target = gmax;
    }
    if (target > p->n) target = p->n;
    P.rows_per_wg = (p->n + target - 1) / target;
    P.G = (int32_t)((p->n + P.rows_per_wg - 1) / P.rows_per_wg);
    if (P.persistent) {
        P.fin_cols = (int32_t)round_up((p->m + P.G - 1) / P.G, 4);
        if (P.fin_cols > s.wg)
            return fail(UOT_ERR_UNSUPPORTED, "persistent loop needs m <= workgroup size * grid (m=%lld, grid=%d)",
                        (long long)p->m, P.G);
        P.lds_bytes = (size_t)P.scratch_bytes + 2 * sizeof(double) * (size_t)P.rows_per_wg;
        if (persist_max_grid(P.k_dtype, P.acc64, P.shape, P.lds_bytes) < P.G)
            return fail(UOT_ERR_UNSUPPORTED, "grid of %d workgroups cannot be co-resident", P.G);
    } else {
        P.lds_bytes = 2 * sizeof(double) * (size_t)P.rows_per_wg + (s.vlds ? (size_t)P.ldv_bytes : 0) + 1024;
    }
    if ((int64_t)P.lds_bytes > max_lds_bytes())
        return fail(UOT_ERR_UNSUPPORTED, "launch shape %d needs %zu bytes of LDS", P.shape, P.lds_bytes);
    P.build_k = (p->K == nullptr);
    P.ldk_ws = round_up(p->m, 64);
    const size_t acc_size = P.acc64 ? 8 : 4;
    size_t off = 0;
    P.off_ctrl = off; off = align_up(off + sizeof(Ctrl), kAlign);
    P.off_cprev = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_w = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_s = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.fin_blocks = P.persistent ? P.G : finalize_blocks(p->m);
    P.off_bp = off; off = align_up(off + sizeof(double) * 2 * (size_t)P.fin_blocks, kAlign);
    P.off_part = off; off = align_up(off + acc_size * (size_t)P.G * P.ldp, kAlign);
    P.off_k = off;
    if (P.build_k) off = align_up(off + (size_t)elem_size(p->k_dtype) * p->n * P.ldk_ws, kAlign);
    P.total = off;
    return UOT_OK;
}

double fi_of(double eps, double tau) { return isinf(tau) ? 1.0 : tau / (tau + eps); }

uot_status run_sinkhorn(const uot_problem* p, const uot_options* o, const uot_outputs* out, void* ws,
                        size_t ws_bytes, hipStream_t stream, uot_profile* prof) {
    Plan P;
    uot_status st = make_plan(p, o, P);
    if (st != UOT_OK) return st;
    if (!out || !out->u || !out->v) return fail(UOT_ERR_ARG, "outputs u and v are required");
    if (!aligned(out->u, 8) || !aligned(out->v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if (ws_bytes < P.total || (P.total > 0 && !ws))
        return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    uint32_t* flag_host = nullptr;
    if (o->tol > 0.0) {
        flag_host = pinned_flag();
        if (!flag_host) return hip_fail(g_pinned_err, "hipHostMalloc");
    }

    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* cprev = (double*)(base + P.off_cprev);
    double* wbuf = (double*)(base + P.off_w);
    double* sbuf = (double*)(base + P.off_s);
    double* bp = (double*)(base + P.off_bp);
    void* part = base + P.off_part;
    const void* K = p->K;
    int64_t ldk = p->ldk;
    if (P.build_k) {
        K = base + P.off_k;
        ldk = P.ldk_ws;
        UOT_HIP(launch_kernel_build(p->C, p->ldc, p->n, p->m, p->eps, nullptr, nullptr, p->k_dtype,
                                    (void*)K, ldk, stream),
                "kernel build");
    }

    const double fi = fi_of(p->eps, p->tau);
    UOT_HIP(launch_init(out->u, p->n, o->u0, out->v, p->m, o->v0, cprev, ctrl, stream), "init");

    PassLaunch L;
    memset(&L, 0, sizeof(L));
    L.K = K;
    L.ldk = ldk;
    L.n = p->n;
    L.m = p->m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.v = out->v;
    L.a = p->a;
    L.u = out->u;
    L.s_out = sbuf;
    L.partials = part;
    L.ldp = P.ldp;
    L.fi = fi;
    L.fi_is_one = (fi == 1.0);
    L.fpot = nullptr;
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.check_done = 1;
    L.ldv_bytes = P.ldv_bytes;

    FinLaunch F;
    memset(&F, 0, sizeof(F));
    F.partials = part;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = p->m;
    F.b = p->b;
    F.v = out->v;
    F.w_out = wbuf;
    F.cprev = cprev;
    F.fi = fi;
    F.fi_is_one = (fi == 1.0);
    F.inv_eps = 1.0 / p->eps;
    F.ctrl = ctrl;
    F.blockpart = bp;
    F.acc64 = P.acc64;

    const int check_every = o->check_every > 0 ? o->check_every : 1;
    const bool fused = o->fused != 0;
    L.test_stop = 0;
    L.fin_blocks = finalize_blocks(p->m);
    L.blockpart = bp;
    L.tol = o->tol;

    // Profiling: events around every launch of sampled iterations
    // (t % kProfileStride == 0) plus the whole loop; unsampled iterations run
    // exactly as without profiling.
    constexpr int kProfileStride = 8;
    enum { K_FUSED = 0, K_ROW = 1, K_COL = 2, K_FIN = 3 };
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    const int per_iter = fused ? 2 : 3;
    size_t evi = 0;
    if (prof) {
        memset(prof, 0, sizeof(*prof));
        size_t sampled = (size_t)(o->max_iter + kProfileStride - 1) / kProfileStride + 1;
        UOT_HIP(events(2 * per_iter * sampled + 2, ev), "hipEventCreate");
        UOT_HIP(hipEventRecord(ev[evi++], stream), "hipEventRecord");
    }
    bool sample = false;
    auto timed = [&](int kind, auto&& launch) -> hipError_t {
        if (sample) {
            ev_kind.push_back(kind);
            hipError_t e = hipEventRecord(ev[evi++], stream);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch();
        if (e != hipSuccess) return e;
        if (sample) return hipEventRecord(ev[evi++], stream);
        return hipSuccess;
    };

    L.fin_blocks = P.fin_blocks;
    int64_t iters_run = 0;
    if (P.persistent && o->max_iter > 0) {
        PersistLaunch PL;
        memset(&PL, 0, sizeof(PL));
        PL.L = L;
        PL.L.check_done = 0;
        PL.F = F;
        PL.max_iter = o->max_iter;
        PL.fin_cols = P.fin_cols;
        PL.scratch_bytes = P.scratch_bytes;
        sample = prof != nullptr;
        UOT_HIP(timed(K_FUSED, [&] { return launch_persist(P.k_dtype, P.acc64, P.shape, PL, P.lds_bytes, stream); }),
                "persistent loop");
        iters_run = o->max_iter;
    }
    for (int t = 0; t < (P.persistent ? 0 : o->max_iter); ++t) {
        sample = prof && (t % kProfileStride == 0);
        L.iter = t + 1;
        PassLaunch L1 = L;
        L1.test_stop = 1;       // the first pass of an iteration applies the stopping test
        if (fused) {
            UOT_HIP(timed(K_FUSED, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_FUSED, P.shape, L1, stream); }),
                    "fused pass");
        } else {
            UOT_HIP(timed(K_ROW, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_ROW, P.shape, L1, stream); }),
                    "row pass");
            UOT_HIP(timed(K_COL, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_COL, P.shape, L, stream); }),
                    "column pass");
        }
        UOT_HIP(timed(K_FIN, [&] { return launch_finalize(F, stream); }), "column finalize");
        iters_run = t + 1;
        // Iteration t+1's first pass decides whether iteration t met tol, so a
        // stop is seen here one check later; the extra launches return at once.
        if (flag_host && (t + 1) % check_every == 0 && t + 1 < o->max_iter) {
            UOT_HIP(hipMemcpyAsync(flag_host, &ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                    "flag copy");
            UOT_HIP(hipStreamSynchronize(stream), "flag sync");
            if (*(volatile uint32_t*)flag_host) break;
        }
    }
    sample = false;
    if (prof) UOT_HIP(hipEventRecord(ev[evi++], stream), "hipEventRecord");

    // Marginals of the final scalings: s = K v_T and w = K^T u_T in one pass.
    PassLaunch LM = L;
    LM.check_done = 0;
    UOT_HIP(launch_pass(P.k_dtype, P.acc64, MODE_MARG, P.shape, LM, stream), "marginal pass");
    FinLaunch FM = F;
    FM.marginal_only = 1;
    FM.c_out = nullptr;
    UOT_HIP(launch_finalize(FM, stream), "marginal finalize");

    ObjLaunch O;
    memset(&O, 0, sizeof(O));
    O.u = out->u;
    O.v = out->v;
    O.s = sbuf;
    O.w = wbuf;
    O.a = p->a;
    O.b = p->b;
    O.n = p->n;
    O.m = p->m;
    O.eps = p->eps;
    O.tau = p->tau;
    O.tau_inf = isinf(p->tau) ? 1 : 0;
    O.r_out = out->r;
    O.c_out = out->c;
    O.loss = out->loss;
    O.info = out->info;
    O.ctrl = ctrl;
    O.tol = o->tol;
    O.iters_run = iters_run;
    O.blockpart = bp;
    O.fin_blocks = P.fin_blocks;
    UOT_HIP(launch_objective(O, stream), "objective");

    if (prof) {
        UOT_HIP(hipStreamSynchronize(stream), "profile sync");
        for (size_t q = 0; q < ev_kind.size(); ++q) {
            float ms = 0.f;
            UOT_HIP(hipEventElapsedTime(&ms, ev[1 + 2 * q], ev[2 + 2 * q]), "hipEventElapsedTime");
            switch (ev_kind[q]) {
                case K_FUSED: prof->fused_launches++; prof->fused_ms += ms; break;
                case K_ROW: prof->row_launches++; prof->row_ms += ms; break;
                case K_COL: prof->col_launches++; prof->col_ms += ms; break;
                default: prof->finalize_launches++; prof->finalize_ms += ms; break;
            }
        }
        UOT_HIP(hipEventElapsedTime(&prof->loop_ms, ev[0], ev[evi - 1]), "hipEventElapsedTime");
    }
    return UOT_OK;
}

}  // namespace

extern "C" {

const char* uot_status_string(uot_status s) {
    switch (s) {
        case UOT_OK: return "ok";
        case UOT_ERR_ARG: return "invalid argument";
        case UOT_ERR_DTYPE: return "unsupported dtype";
        case UOT_ERR_ALIGN: return "misaligned pointer or leading dimension";
        case UOT_ERR_WORKSPACE: return "workspace too small";
        case UOT_ERR_UNSUPPORTED: return "unsupported configuration";
        case UOT_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* uot_last_error(void) { return g_last_error.c_str(); }

size_t uot_cost_workspace_size(int64_t n, int64_t m) {
    if (n < 1 || m < 1) return 0;
    return align_up(sizeof(double) * (size_t)(cost_blocks(n, m) + 1), kAlign);
}

uot_status uot_cost_from_points(const double* x, const double* y, int64_t n, int64_t m, int64_t d,
                                int32_t kind, int32_t normalize_max, double* C, int64_t ldc, void* ws,
                                size_t ws_bytes, void* stream) {
    if (n < 1 || m < 1 || d < 1) return fail(UOT_ERR_ARG, "n, m, d must be >= 1");
    if (!x || !y || !C) return fail(UOT_ERR_ARG, "x, y, C must not be NULL");
    if (kind != UOT_COST_SQEUCLID && kind != UOT_COST_COSINE) return fail(UOT_ERR_ARG, "unknown cost kind %d", kind);
    if (ldc < m) return fail(UOT_ERR_ARG, "ldc < m");
    if (!aligned(x, 8) || !aligned(y, 8) || !aligned(C, 8)) return fail(UOT_ERR_ALIGN, "x, y, C must be 8-byte aligned");
    size_t need = uot_cost_workspace_size(n, m);
    if (!ws || ws_bytes < need) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
    UOT_HIP(launch_cost(x, y, n, m, d, kind, normalize_max, C, ldc, (double*)ws, (hipStream_t)stream), "cost");
    return UOT_OK;
}

uot_status uot_kernel_from_cost(const double* C, int64_t ldc, int64_t n, int64_t m, double eps, const double* f,
                                const double* g, int32_t k_dtype, void* K, int64_t ldk, void* stream) {
    if (n < 1 || m < 1) return fail(UOT_ERR_ARG, "n, m must be >= 1");
    if (!C || !K) return fail(UOT_ERR_ARG, "C and K must not be NULL");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (ldc < m || ldk < m) return fail(UOT_ERR_ARG, "leading dimensions must be >= m");
    if (k_dtype != UOT_F64 && k_dtype != UOT_F32) return fail(UOT_ERR_DTYPE, "K dtype %d not supported here", k_dtype);
    int vec = 16 / elem_size(k_dtype);
    if (!aligned(K, 16) || ldk % vec != 0) return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned, ldk a multiple of %d", vec);
    if (!aligned(C, 8)) return fail(UOT_ERR_ALIGN, "C must be 8-byte aligned");
    UOT_HIP(launch_kernel_build(C, ldc, n, m, eps, f, g, k_dtype, K, ldk, (hipStream_t)stream), "kernel build");
    return UOT_OK;
}

size_t uot_sinkhorn_workspace_size(const uot_problem* prob, const uot_options* opt) {
    Plan P;
    if (make_plan(prob, opt, P) != UOT_OK) return 0;
    return P.total;
}

uot_status uot_sinkhorn(const uot_problem* prob, const uot_options* opt, const uot_outputs* out, void* ws,
                        size_t ws_bytes, void* stream) {
    return run_sinkhorn(prob, opt, out, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

uot_status uot_sinkhorn_profiled(const uot_problem* prob, const uot_options* opt, const uot_outputs* out,
                                 void* ws, size_t ws_bytes, void* stream, uot_profile* prof) {
    if (!prof) return fail(UOT_ERR_ARG, "prof must not be NULL");
    return run_sinkhorn(prob, opt, out, ws, ws_bytes, (hipStream_t)stream, prof);
}

}  // extern "C"
