// C-ABI of libuot.so: argument checks, workspace layout, launch sequence.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "multi.h"
#include "online.h"
#include "lse.h"
#include "plan.h"
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

// Pinned host words through which the host reads the stop flag and the
// absorption maxima.  Each call that reads them takes a slot of its own from
// a pool (grown on demand, kept for the process) and returns it when it
// ends, so concurrent calls on different streams or threads never share one.
struct PinnedSlot {
    uint32_t* p = nullptr;   // 64 bytes: flag word at 0, two doubles at byte 16
    uint32_t* flag() const { return p; }
    double* vals() const { return (double*)(p + 4); }
};
std::mutex g_pin_mu;
std::vector<uint32_t*> g_pin_free;

hipError_t pinned_acquire(PinnedSlot& s) {
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        if (!g_pin_free.empty()) {
            s.p = g_pin_free.back();
            g_pin_free.pop_back();
            return hipSuccess;
        }
    }
    return hipHostMalloc((void**)&s.p, 64, hipHostMallocDefault);
}

void pinned_release(PinnedSlot& s) {
    if (!s.p) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(s.p);
    s.p = nullptr;
}

struct PinnedGuard {
    PinnedSlot slot;
    ~PinnedGuard() { pinned_release(slot); }
};

// Events of profiled runs: taken from a pool per call and returned at its end.
std::mutex g_ev_mu;
std::vector<hipEvent_t> g_ev_free;

hipError_t events_acquire(size_t count, std::vector<hipEvent_t>& out) {
    out.clear();
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        while (out.size() < count && !g_ev_free.empty()) {
            out.push_back(g_ev_free.back());
            g_ev_free.pop_back();
        }
    }
    while (out.size() < count) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        out.push_back(e);
    }
    return hipSuccess;
}

struct EventGuard {
    std::vector<hipEvent_t> ev;
    ~EventGuard() {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        g_ev_free.insert(g_ev_free.end(), ev.begin(), ev.end());
    }
};

// Scratch of the no-allocation entry point (uot_sinkhorn_noalloc): one copy
// per GPU, held until the process ends, shared by every such call on that
// GPU.  Its host-side name is not a device address: host code uses only the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)UOT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
bool g_scratch_ready[kMaxDevices];

// Device address of the current device's scratch (looked up once per device).
uot_status scratch_for_current_device(void** ptr);

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
    bool stab;            // log-domain absorption (state u, v, f, g in the workspace)
    // workspace offsets
    size_t off_ctrl, off_cprev, off_w, off_s, off_bp, off_part, off_k, off_stab, total;
};

// Options that record the forward's iterates (checkpoints or every iterate),
// which only the single-problem stored-kernel loop supports.
bool records_iterates(const uot_options* o) { return o->checkpoint_every != 0 || o->store_iterates != 0; }

uot_status check_problem(const uot_problem* p, const uot_options* o) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "empty problem (n=%lld, m=%lld)", (long long)p->n, (long long)p->m);
    if (!p->a || !p->b) return fail(UOT_ERR_ARG, "a and b must not be NULL");
    if (!aligned(p->a, 8) || !aligned(p->b, 8)) return fail(UOT_ERR_ALIGN, "a and b must be 8-byte aligned");
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "tau must be > 0 (or +inf)");
    if (o->max_iter < 0) return fail(UOT_ERR_ARG, "max_iter must be >= 0");
    if (o->absorb_log_threshold < 0.0 || !(o->absorb_log_threshold == o->absorb_log_threshold))
        return fail(UOT_ERR_ARG, "absorb_log_threshold must be >= 0");
    const bool stab = o->absorb_log_threshold > 0.0;
    if (stab && !p->C) return fail(UOT_ERR_ARG, "log-domain absorption rebuilds K from C: C is required");
    if (stab && (o->persistent || o->checkpoint_every > 0))
        return fail(UOT_ERR_UNSUPPORTED, "log-domain absorption runs with per-iteration launches and no checkpoints");
    if (o->checkpoint_every < 0) return fail(UOT_ERR_ARG, "checkpoint_every must be >= 0");
    if (o->checkpoint_every > 0 && (o->tol > 0.0 || o->persistent))
        return fail(UOT_ERR_UNSUPPORTED, "checkpoints need a fixed iteration count (tol <= 0) and per-iteration launches");
    if (o->store_iterates != 0 && o->store_iterates != 1) return fail(UOT_ERR_ARG, "store_iterates must be 0 or 1");
    if (o->store_iterates && (o->checkpoint_every != 0 || o->tol > 0.0 || o->persistent || stab))
        return fail(UOT_ERR_UNSUPPORTED,
                    "stored iterates need checkpoint_every = 0, a fixed iteration count (tol <= 0), per-iteration "
                    "launches and no absorption");
    if (p->k_dtype != UOT_F64 && p->k_dtype != UOT_F32 && p->k_dtype != UOT_BF16 && p->k_dtype != UOT_FP8_E4M3)
        return fail(UOT_ERR_DTYPE, "K dtype %d not supported", (int)p->k_dtype);
    if ((p->k_dtype == UOT_BF16 || p->k_dtype == UOT_FP8_E4M3) && (!o->fused || o->persistent))
        return fail(UOT_ERR_UNSUPPORTED, "BF16 and FP8 K run the fused per-iteration pass only");
    if (!(p->k_scale >= 0.0) || !isfinite(p->k_scale)) return fail(UOT_ERR_ARG, "k_scale must be finite and >= 0");
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

int default_shape(int64_t nv, bool persistent, int k_dtype, bool acc64) {
    // Smallest shape in the storage type's list whose lanes cover a row (in
    // 16-byte chunks); rows of up to 2048 chunks go in batches of rows per
    // barrier (the persistent loop instantiates the one-row shapes only).
    // The 512-lane batched shapes 12-14 were measured fastest for rows of
    // 8192 FP32, BF16 and FP8 entries (eight waves per barrier instead of
    // sixteen, twice the bytes per lane in flight).
    static const int order_f32[] = {11, 10, 9, 12, 6};
    static const int order_bf16[] = {11, 10, 13, 8, 6};
    static const int order_fp8[] = {11, 14, 9, 8, 6};
    static const int order_other[] = {11, 10, 9, 8, 6};
    static const int order_one_row[] = {0, 1, 2, 3, 4, 6};
    const int* order = order_other;
    if (persistent) {
        for (int idx : order_one_row)
            if ((int64_t)pass_shape(idx).wg * pass_shape(idx).nc >= nv) return idx;
        return -1;
    }
    if (k_dtype == UOT_F32 && !acc64) order = order_f32;
    else if (k_dtype == UOT_BF16) order = order_bf16;
    else if (k_dtype == UOT_FP8_E4M3) order = order_fp8;
    for (int q = 0; q < 5; ++q)
        if ((int64_t)pass_shape(order[q]).wg * pass_shape(order[q]).nc >= nv) return order[q];
    return -1;
}

// Largest dynamic LDS one workgroup may use on the current device.
int64_t max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

// Compute units of the current device (256 when it cannot be queried).
int64_t cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

uot_status make_plan(const uot_problem* p, const uot_options* o, Plan& P, bool one_row = false) {
    uot_status st = check_problem(p, o);
    if (st != UOT_OK) return st;
    P.k_dtype = p->k_dtype;
    P.acc64 = (p->k_dtype == UOT_F64) || (p->k_dtype == UOT_F32 && o->accum == UOT_ACC_F64);
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
        P.shape = default_shape(nv, o->persistent != 0 || one_row, P.k_dtype, P.acc64);
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
    if (P.persistent && (s.rb != 1 || P.shape > 7))
        return fail(UOT_ERR_UNSUPPORTED, "the persistent loop runs the one-row shapes (0-7) only");
    int64_t target = 256LL * (1024 / s.wg);     // about one wave of workgroups on 256 CUs
    if (!P.persistent) {
        // Shapes whose registers allow fewer than 1024 lanes per CU: the
        // grid above runs in several rounds of resident workgroups.  That
        // pays only while each strip is long (measured: 2 MiB and 4 MiB
        // strips gain from two rounds, 0.5 MiB and 1 MiB strips lose); with
        // shorter strips the grid is cut to one round.
        const size_t lds_est = (s.vlds ? (size_t)P.ldv_bytes : 0) + 2 * sizeof(double) * (size_t)((p->n + 255) / 256);
        int dev = 0, cus = 0;
        const int per_cu = pass_resident_per_cu(P.k_dtype, P.acc64, MODE_FUSED, P.shape, lds_est);
        const int64_t strip_bytes = (p->n + target - 1) / target * p->m * elem_size(p->k_dtype);
        if (per_cu > 0 && strip_bytes < (2LL << 20) && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            target = std::min<int64_t>(target, (int64_t)per_cu * cus);
    }
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
    // A strip's loads use 32-bit byte offsets from its first row, including
    // the rows prefetched past its end.
    {
        const int64_t ldk_eff = p->K ? p->ldk : round_up(p->m, 64);
        if ((P.rows_per_wg + 16) * ldk_eff * elem_size(p->k_dtype) >= (int64_t)1 << 31)
            return fail(UOT_ERR_UNSUPPORTED, "a strip of %lld rows with ldk=%lld spans 2 GiB or more",
                        (long long)P.rows_per_wg, (long long)ldk_eff);
    }
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
    P.stab = o->absorb_log_threshold > 0.0;
    P.build_k = (p->K == nullptr) || P.stab;
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
    P.off_stab = off;
    if (P.stab) off = align_up(off + sizeof(double) * (2 * (size_t)p->n + 3 * (size_t)p->m + 4), kAlign);
    P.total = off;
    return UOT_OK;
}

double fi_of(double eps, double tau) { return isinf(tau) ? 1.0 : tau / (tau + eps); }

// Level of the absorption check after a rebuild that left the residue `res`
// (max |log u|, |log v|): the threshold, or res plus half the threshold when
// the residue is beyond it, never above kAbsorbCeiling (unless the threshold
// itself is).
constexpr double kAbsorbCeiling = 60.0;
double absorb_level(double res, double thr) {
    if (!(res > thr)) return thr;
    return std::max(thr, std::min(res + 0.5 * thr, kAbsorbCeiling));
}

// no_sync: never wait on the stream (the caller may not allow it): with
// tol > 0 every iteration up to max_iter is enqueued and the launches after
// the stop return at once; absorption, which decides on the host, is refused.
uot_status run_sinkhorn(const uot_problem* p, const uot_options* o, const uot_outputs* out, void* ws,
                        size_t ws_bytes, hipStream_t stream, uot_profile* prof, bool no_sync = false) {
    Plan P;
    uot_status st = make_plan(p, o, P);
    if (st != UOT_OK) return st;
    if (!out || !out->u || !out->v) return fail(UOT_ERR_ARG, "outputs u and v are required");
    if (!aligned(out->u, 8) || !aligned(out->v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if (ws_bytes < P.total || (P.total > 0 && !ws))
        return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    if (no_sync && (P.stab || prof))
        return fail(UOT_ERR_UNSUPPORTED, "absorption and profiling wait on the stream");
    PinnedGuard pin;
    if ((o->tol > 0.0 && !no_sync) || P.stab) UOT_HIP(pinned_acquire(pin.slot), "hipHostMalloc");
    uint32_t* flag_host = (o->tol > 0.0 && !no_sync) ? pin.slot.flag() : nullptr;

    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* cprev = (double*)(base + P.off_cprev);
    double* wbuf = (double*)(base + P.off_w);
    double* sbuf = (double*)(base + P.off_s);
    double* bp = (double*)(base + P.off_bp);
    void* part = base + P.off_part;
    const void* K = p->K;
    int64_t ldk = p->ldk;
    // FP8 stores 448 K (its largest finite value maps to the row maximum 1).
    const double store_scale = (p->k_dtype == UOT_FP8_E4M3) ? 448.0 : 1.0;
    double k_scale = (p->K && p->k_scale > 0.0) ? p->k_scale : 1.0;
    if (P.build_k) {
        K = base + P.off_k;
        ldk = P.ldk_ws;
        k_scale = 1.0 / store_scale;
    }
    // Scaling state: the outputs themselves, or (with absorption) workspace
    // vectors u, v next to the potentials f, g; the outputs then get the totals.
    double* su = out->u;
    double* sv = out->v;
    double* fpot = nullptr;
    double* gpot = nullptr;
    double* absorb_vals = nullptr;
    double* gmin_scratch = nullptr;
    if (P.stab) {
        double* sb = (double*)(base + P.off_stab);
        su = sb;
        sv = su + p->n;
        fpot = sv + p->m;
        gpot = fpot + p->n;
        absorb_vals = gpot + p->m;
        gmin_scratch = absorb_vals + 4;
    }
    if (P.build_k && !P.stab)
        UOT_HIP(launch_kernel_build(p->C, p->ldc, p->n, p->m, p->eps, nullptr, nullptr, p->k_dtype, (void*)K, ldk,
                                    store_scale, stream),
                "kernel build");

    const double fi = fi_of(p->eps, p->tau);
    UOT_HIP(launch_init(su, p->n, o->u0, sv, p->m, o->v0, cprev, ctrl, stream), "init");
    int32_t absorptions = 0;
    double arm = o->absorb_log_threshold;   // level the absorption check compares against
    double* host_vals = nullptr;
    if (P.stab) {
        // g = 0 (zeroed through the init kernel's cprev path is not available: reuse it on g)
        UOT_HIP(launch_init(nullptr, 0, nullptr, nullptr, p->m, nullptr, gpot, ctrl, stream), "init");
        UOT_HIP(launch_rebuild(p->C, p->ldc, p->n, p->m, p->eps, fpot, gpot, su, sv, gmin_scratch, p->k_dtype,
                               (void*)K, ldk, store_scale, 1, stream),
                "kernel rebuild");
        host_vals = pin.slot.vals();
    }
    // Checkpoint slot c holds v and K^T u after iteration c*k (slot 0: the start v).
    const int ck = o->checkpoint_every;
    if (ck > 0) {
        if (!out->ckpt) return fail(UOT_ERR_ARG, "checkpoint_every > 0 needs outputs->ckpt");
        UOT_HIP(hipMemcpyAsync(out->ckpt, out->v, sizeof(double) * p->m, hipMemcpyDeviceToDevice, stream),
                "checkpoint copy");
    }
    // Stored iterates: iteration t reads v_{t-1} and writes u_t, its row sums,
    // v_t and K^T u_t straight into the record (blocks V, W, U, S).
    const bool store = o->store_iterates != 0;
    double *tr_v = nullptr, *tr_w = nullptr, *tr_u = nullptr, *tr_s = nullptr;
    if (store && o->max_iter > 0) {
        if (!out->ckpt) return fail(UOT_ERR_ARG, "store_iterates needs outputs->ckpt");
        if (!aligned(out->ckpt, 8)) return fail(UOT_ERR_ALIGN, "ckpt must be 8-byte aligned");
        const size_t T = (size_t)o->max_iter;
        tr_v = out->ckpt;
        tr_w = tr_v + (T + 1) * p->m;
        tr_u = tr_w + T * p->m;
        tr_s = tr_u + T * p->n;
        UOT_HIP(hipMemcpyAsync(tr_v, sv, sizeof(double) * p->m, hipMemcpyDeviceToDevice, stream), "iterate copy");
    }

    PassLaunch L;
    memset(&L, 0, sizeof(L));
    L.K = K;
    L.ldk = ldk;
    L.n = p->n;
    L.m = p->m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.v = sv;
    L.a = p->a;
    L.u = su;
    L.s_out = sbuf;
    L.partials = part;
    L.ldp = P.ldp;
    L.fi = fi;
    L.fi_is_one = (fi == 1.0);
    L.fpot = fpot;
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.check_done = 1;
    L.ldv_bytes = P.ldv_bytes;
    L.k_scale = k_scale;

    FinLaunch F;
    memset(&F, 0, sizeof(F));
    F.partials = part;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = p->m;
    F.b = p->b;
    F.v = sv;
    F.w_out = wbuf;
    F.cprev = cprev;
    F.gpot = gpot;
    F.k_scale = k_scale;
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
    EventGuard evg;
    std::vector<hipEvent_t>& ev = evg.ev;
    std::vector<int> ev_kind;
    const int per_iter = fused ? 2 : 3;
    size_t evi = 0;
    if (prof) {
        memset(prof, 0, sizeof(*prof));
        size_t sampled = (size_t)(o->max_iter + kProfileStride - 1) / kProfileStride + 1;
        UOT_HIP(events_acquire(2 * per_iter * sampled + 2, ev), "hipEventCreate");
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
        FinLaunch F1 = F;
        if (store) {
            L1.v = tr_v + (size_t)t * p->m;
            L1.u = tr_u + (size_t)t * p->n;
            L1.s_trace = tr_s + (size_t)t * p->n;
            F1.v = tr_v + (size_t)(t + 1) * p->m;
            F1.w_out = tr_w + (size_t)t * p->m;
        }
        PassLaunch L2 = L1;     // the column pass of the unfused form
        L1.test_stop = 1;       // the first pass of an iteration applies the stopping test
        L2.s_trace = nullptr;
        if (fused) {
            UOT_HIP(timed(K_FUSED, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_FUSED, P.shape, L1, stream); }),
                    "fused pass");
        } else {
            UOT_HIP(timed(K_ROW, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_ROW, P.shape, L1, stream); }),
                    "row pass");
            UOT_HIP(timed(K_COL, [&] { return launch_pass(P.k_dtype, P.acc64, MODE_COL, P.shape, L2, stream); }),
                    "column pass");
        }
        UOT_HIP(timed(K_FIN, [&] { return launch_finalize(F1, stream); }), "column finalize");
        iters_run = t + 1;
        if (P.stab && (t + 1) % check_every == 0 && t + 1 < o->max_iter) {
            // Absorb when a scaling's log leaves [-threshold, threshold] (above
            // the current level): v goes into g, then f and Kt are rebuilt from C
            // (u keeps its total).
            UOT_HIP(launch_absorb_check(su, p->n, sv, p->m, absorb_vals, stream), "absorb check");
            UOT_HIP(hipMemcpyAsync(host_vals, absorb_vals, 2 * sizeof(double), hipMemcpyDeviceToHost, stream),
                    "absorb copy");
            UOT_HIP(hipStreamSynchronize(stream), "absorb sync");
            if (std::max(host_vals[0], host_vals[1]) > arm) {
                UOT_HIP(launch_absorb_apply(sv, gpot, p->m, p->eps, stream), "absorb");
                UOT_HIP(launch_rebuild(p->C, p->ldc, p->n, p->m, p->eps, fpot, gpot, su, sv, gmin_scratch,
                                       p->k_dtype, (void*)K, ldk, store_scale, 0, stream),
                        "kernel rebuild");
                ++absorptions;
                // What the normalisation puts back (every row and column of Kt
                // at maximum 1) cannot be absorbed: when that residue is beyond
                // the threshold, the next absorption waits until the scalings
                // grow by half a threshold more (at most to kAbsorbCeiling,
                // inside the FP32 range of the passes' lane products).
                UOT_HIP(launch_absorb_check(su, p->n, sv, p->m, absorb_vals, stream), "absorb check");
                UOT_HIP(hipMemcpyAsync(host_vals, absorb_vals, 2 * sizeof(double), hipMemcpyDeviceToHost, stream),
                        "absorb copy");
                UOT_HIP(hipStreamSynchronize(stream), "absorb sync");
                arm = absorb_level(std::max(host_vals[0], host_vals[1]), o->absorb_log_threshold);
            }
        }
        if (ck > 0 && (t + 1) % ck == 0 && t + 1 < o->max_iter) {
            double* slot = out->ckpt + (size_t)((t + 1) / ck) * 2 * p->m;
            UOT_HIP(hipMemcpyAsync(slot, out->v, sizeof(double) * p->m, hipMemcpyDeviceToDevice, stream),
                    "checkpoint copy");
            UOT_HIP(hipMemcpyAsync(slot + p->m, wbuf, sizeof(double) * p->m, hipMemcpyDeviceToDevice, stream),
                    "checkpoint copy");
        }
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
    if (store && iters_run > 0) {
        UOT_HIP(hipMemcpyAsync(su, tr_u + (size_t)(iters_run - 1) * p->n, sizeof(double) * p->n,
                               hipMemcpyDeviceToDevice, stream),
                "iterate copy");
        UOT_HIP(hipMemcpyAsync(sv, tr_v + (size_t)iters_run * p->m, sizeof(double) * p->m, hipMemcpyDeviceToDevice,
                               stream),
                "iterate copy");
    }

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
    O.u = su;
    O.v = sv;
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
    O.fpot = fpot;
    O.gpot = gpot;
    O.f_out = out->f;
    O.g_out = out->g;
    O.u_tot = P.stab ? out->u : nullptr;
    O.v_tot = P.stab ? out->v : nullptr;
    O.absorptions = absorptions;
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

uot_status scratch_for_current_device(void** ptr) {
    int dev = 0;
    UOT_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(UOT_ERR_UNSUPPORTED, "device index %d (at most %d devices)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ready[dev]) {
        void* p = nullptr;
        UOT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p || !aligned(p, kAlign)) return fail(UOT_ERR_HIP, "scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = p;
        g_scratch_ready[dev] = true;
    }
    *ptr = g_scratch_ptr[dev];
    return UOT_OK;
}

// ---------------------------------------------------------------------------
// Reverse pass driver
// ---------------------------------------------------------------------------
struct BwdPlan {
    Plan F;                   // forward plan (recompute and the column pass)
    int nc;                   // adjoint chunks per lane
    int64_t rows_per_wg;
    int32_t G;
    int32_t dim;
    int k, nseg;
    bool stored;              // the forward stored every iterate: no recompute
    bool cost_grad;           // store the factors of Kbar for dL/dC or dL/dy
    int64_t nterms;           // 2T + 2, padded to a multiple of kGradcSlotPad
    int64_t ldl, ldr;         // n and m padded to kGradcRowPad (factor row lengths)
    int32_t row_tiles;        // row tiles of the cost-gradient product
    size_t off_fwd, off_part, off_str, off_utr, off_wtr, off_vtr, off_useed, off_abar, off_gsum, off_gy,
        off_bbar, off_cbar, off_wfin, off_avec, off_lf, off_rf, off_ysum, total;
};

uot_status make_bwd_plan(const uot_problem* p, const uot_options* o, int64_t dim, bool cost_grad, BwdPlan& B) {
    uot_options fo = *o;
    fo.fused = 1;
    fo.persistent = 0;
    uot_status st = make_plan(p, &fo, B.F);
    if (st != UOT_OK) return st;
    if (o->max_iter < 1) return fail(UOT_ERR_ARG, "the reverse pass needs max_iter >= 1");
    if (o->store_iterates ? o->checkpoint_every != 0 : o->checkpoint_every < 1)
        return fail(UOT_ERR_ARG, "the reverse pass needs checkpoint_every >= 1 or stored iterates (not both)");
    if (o->tol > 0.0) return fail(UOT_ERR_UNSUPPORTED, "the reverse pass differentiates a fixed iteration count (tol <= 0)");
    if (p->k_dtype != UOT_F32 && p->k_dtype != UOT_F64)
        return fail(UOT_ERR_DTYPE, "the reverse pass runs with FP32 or FP64 K");
    if (dim != 0 && dim != 2 && dim != 3) return fail(UOT_ERR_UNSUPPORTED, "point dimension %lld (0, 2 or 3)", (long long)dim);
    const int64_t nv = (p->m + B.F.vec - 1) / B.F.vec;
    const int awg = adj_wg();
    B.nc = (int)((nv + awg - 1) / awg);
    if (B.nc == 3) B.nc = 4;
    if (B.nc > adj_chunks_max(p->k_dtype))
        return fail(UOT_ERR_UNSUPPORTED, "the reverse pass holds rows of up to %d columns",
                    adj_chunks_max(p->k_dtype) * awg * B.F.vec);
    int64_t target = p->n < 256 ? p->n : 256;
    B.rows_per_wg = (p->n + target - 1) / target;
    B.G = (int32_t)((p->n + B.rows_per_wg - 1) / B.rows_per_wg);
    B.dim = (int32_t)dim;
    B.stored = o->store_iterates != 0;
    B.k = B.stored ? 0 : o->checkpoint_every;      // recompute buffers hold one segment
    B.nseg = B.stored ? 0 : (o->max_iter + B.k - 1) / B.k;
    const int64_t n = p->n, m = p->m;
    const size_t d8 = sizeof(double);
    const size_t acc = (p->k_dtype == UOT_F64) ? 8 : 4;
    size_t off = 0;
    B.off_fwd = off; off = align_up(off + B.F.total, kAlign);
    B.off_part = off; off = align_up(off + acc * (size_t)B.G * B.F.ldp, kAlign);
    B.off_str = off; off = align_up(off + d8 * (size_t)B.k * n, kAlign);
    B.off_utr = off; off = align_up(off + d8 * (size_t)B.k * n, kAlign);
    B.off_wtr = off; off = align_up(off + d8 * (size_t)B.k * m, kAlign);
    B.off_vtr = off; off = align_up(off + d8 * (size_t)B.k * m, kAlign);
    B.off_useed = off; off = align_up(off + d8 * n, kAlign);
    B.off_abar = off; off = align_up(off + d8 * n, kAlign);
    B.off_gsum = off; off = align_up(off + d8 * n, kAlign);
    B.off_gy = off; off = align_up(off + d8 * n * (dim > 0 ? dim : 1), kAlign);
    B.off_bbar = off; off = align_up(off + d8 * m, kAlign);
    B.off_cbar = off; off = align_up(off + d8 * m, kAlign);
    B.off_wfin = off; off = align_up(off + d8 * m, kAlign);
    B.off_avec = off; off = align_up(off + d8 * m, kAlign);
    B.cost_grad = cost_grad;
    B.nterms = round_up(2 * (int64_t)o->max_iter + 2, kGradcSlotPad);
    B.ldl = round_up(n, kGradcRowPad);
    B.ldr = round_up(m, kGradcRowPad);
    B.row_tiles = gradc_row_tiles(n);
    B.off_lf = B.off_rf = B.off_ysum = off;
    if (cost_grad) {
        B.off_lf = off; off = align_up(off + d8 * (size_t)B.nterms * B.ldl, kAlign);
        B.off_rf = off; off = align_up(off + d8 * (size_t)B.nterms * B.ldr, kAlign);
        B.off_ysum = off; off = align_up(off + d8 * (size_t)B.row_tiles * (1 + (dim > 0 ? dim : 0)) * m, kAlign);
    }
    B.total = off;
    return UOT_OK;
}

uot_status run_backward(const uot_problem* p, const uot_options* o, const double* uT, const double* vT,
                        const double* ckpt, const double* grad_loss, double* grad_a, double* grad_b,
                        double* grad_C, int64_t ldgc, const double* x, const double* y, int64_t dim,
                        double* grad_x, double* grad_y, void* ws, size_t ws_bytes, hipStream_t stream) {
    BwdPlan B;
    const bool cost_grad = grad_C != nullptr || grad_y != nullptr;
    uot_status st = make_bwd_plan(p, o, dim, cost_grad, B);
    if (st != UOT_OK) return st;
    if (!uT || !vT || !ckpt || !grad_loss) return fail(UOT_ERR_ARG, "u, v, ckpt and grad_loss are required");
    if (grad_x && (dim == 0 || !x)) return fail(UOT_ERR_ARG, "grad_x needs x and dim > 0");
    if (grad_y && (dim == 0 || !x)) return fail(UOT_ERR_ARG, "grad_y needs x, y and dim > 0");
    if (dim > 0 && !y) return fail(UOT_ERR_ARG, "dim > 0 needs the target points y");
    if (grad_C && ldgc < p->m) return fail(UOT_ERR_ARG, "ldgc (%lld) < m (%lld)", (long long)ldgc, (long long)p->m);
    if ((grad_C && !aligned(grad_C, 8)) || (grad_y && !aligned(grad_y, 8)))
        return fail(UOT_ERR_ALIGN, "grad_C and grad_y must be 8-byte aligned");
    if (ws_bytes < B.total || !ws) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", B.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    const Plan& P = B.F;
    const int64_t n = p->n, m = p->m;
    char* base = (char*)ws;
    char* fw = base + B.off_fwd;
    Ctrl* ctrl = (Ctrl*)(fw + P.off_ctrl);
    double* cprev = (double*)(fw + P.off_cprev);
    double* bp = (double*)(fw + P.off_bp);
    void* fpart = fw + P.off_part;
    double* str = (double*)(base + B.off_str);
    double* utr = (double*)(base + B.off_utr);
    double* wtr = (double*)(base + B.off_wtr);
    double* vtr = (double*)(base + B.off_vtr);
    double* useed = (double*)(base + B.off_useed);
    double* abar = (double*)(base + B.off_abar);
    double* gsum = (double*)(base + B.off_gsum);
    double* gy = (double*)(base + B.off_gy);
    double* bbar = (double*)(base + B.off_bbar);
    double* cbar = (double*)(base + B.off_cbar);
    double* wfin = (double*)(base + B.off_wfin);
    double* avec = (double*)(base + B.off_avec);
    double* Lf = cost_grad ? (double*)(base + B.off_lf) : nullptr;
    double* Rf = cost_grad ? (double*)(base + B.off_rf) : nullptr;
    const int64_t ldl = B.ldl, ldr = B.ldr;
    if (cost_grad) {
        // padding slots and the rows past n (columns past m) hold zero factors
        UOT_HIP(launch_fill_f64(Lf, B.nterms * ldl, 0.0, stream), "factor padding");
        UOT_HIP(launch_fill_f64(Rf, B.nterms * ldr, 0.0, stream), "factor padding");
    }
    const void* K = p->K;
    int64_t ldk = p->ldk;
    if (P.build_k) {
        K = fw + P.off_k;
        ldk = P.ldk_ws;
        UOT_HIP(launch_kernel_build(p->C, p->ldc, n, m, p->eps, nullptr, nullptr, p->k_dtype, (void*)K, ldk, 1.0, stream),
                "kernel build");
    }
    UOT_HIP(launch_init(nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, ctrl, stream), "init");
    const double fi = fi_of(p->eps, p->tau);
    const int tau_inf = isinf(p->tau) ? 1 : 0;

    // Forward pass parameters (recompute and the K^T u_T column pass).
    PassLaunch L;
    memset(&L, 0, sizeof(L));
    L.K = K;
    L.ldk = ldk;
    L.n = n;
    L.m = m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.a = p->a;
    L.partials = fpart;
    L.ldp = P.ldp;
    L.fi = fi;
    L.fi_is_one = (fi == 1.0);
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.ldv_bytes = P.ldv_bytes;
    L.fin_blocks = finalize_blocks(m);
    L.blockpart = bp;
    L.k_scale = 1.0;
    FinLaunch F;
    memset(&F, 0, sizeof(F));
    F.k_scale = 1.0;
    F.partials = fpart;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = m;
    F.b = p->b;
    F.cprev = cprev;
    F.fi = fi;
    F.fi_is_one = (fi == 1.0);
    F.inv_eps = 1.0 / p->eps;
    F.ctrl = ctrl;
    F.blockpart = bp;
    F.acc64 = P.acc64;

    AdjLaunch A;
    memset(&A, 0, sizeof(A));
    A.K = K;
    A.ldk = ldk;
    A.n = n;
    A.m = m;
    A.rows_per_wg = B.rows_per_wg;
    A.grid = B.G;
    A.y = y;
    A.a = p->a;
    A.useed = useed;
    A.abar = abar;
    A.gsum = gsum;
    A.gy = gy;
    A.partials = base + B.off_part;
    A.ldp = P.ldp;
    A.fi = fi;
    A.eps = p->eps;
    A.tau = p->tau;
    A.tau_inf = tau_inf;
    AdjColLaunch Cc;
    memset(&Cc, 0, sizeof(Cc));
    Cc.ldp = P.ldp;
    Cc.m = m;
    Cc.b = p->b;
    Cc.cbar = cbar;
    Cc.bbar = bbar;
    Cc.out = avec;
    Cc.fi = fi;
    Cc.eps = p->eps;
    Cc.tau = p->tau;
    Cc.tau_inf = tau_inf;

    // 1. w_T = K^T u_T (forward column pass), then cbar, bbar and the seed's A = cbar v_T.
    {
        PassLaunch LC = L;
        LC.u = (double*)uT;
        UOT_HIP(launch_pass(P.k_dtype, P.acc64, MODE_COL, P.shape, LC, stream), "column pass");
        AdjColLaunch C1 = Cc;
        C1.partials = fpart;
        C1.G = P.G;
        C1.acc64 = P.acc64;
        C1.mode = ADJ_COL_PREP;
        C1.v = vT;
        C1.w = wfin;
        UOT_HIP(launch_adj_col(C1, stream), "adjoint columns");
    }
    // 2. seed pass, 3. vbar_T and wbar_T
    {
        AdjLaunch S = A;
        S.A = avec;
        S.B = vT;
        S.u = uT;
        if (cost_grad) {
            // slot 0: (rbar u_T) v_T^T, slot 1: u_T (cbar v_T)^T
            S.st_q = Lf;
            S.st_u = Lf + ldl;
            S.st_a = Rf + ldr;
            S.st_b = Rf;
        }
        UOT_HIP(launch_adj(p->k_dtype, B.nc, ADJ_SEED, (int)dim, S, stream), "adjoint seed pass");
        AdjColLaunch C2 = Cc;
        C2.partials = A.partials;
        C2.G = B.G;
        C2.acc64 = (p->k_dtype == UOT_F64);
        C2.mode = ADJ_COL_SEED;
        C2.v = vT;
        C2.w = wfin;
        UOT_HIP(launch_adj_col(C2, stream), "adjoint columns");
    }
    // 4. reverse steps t = T .. 1 over the iterates: read from the forward's
    // record, or recomputed segment by segment (newest first) from checkpoints.
    const int T = o->max_iter;
    auto reverse_step = [&](int t, const double* vprev, const double* ut, const double* st,
                            const double* wprev) -> uot_status {
        AdjLaunch S = A;
        S.A = avec;
        S.B = vprev;
        S.u = ut;
        S.s = st;
        S.add_seed = (t == T) ? 1 : 0;
        if (cost_grad) {
            // slot 2t: u_t wbar_t^T, slot 2t + 1: sbar_t v_{t-1}^T
            S.st_u = Lf + (int64_t)(2 * t) * ldl;
            S.st_q = Lf + (int64_t)(2 * t + 1) * ldl;
            S.st_a = Rf + (int64_t)(2 * t) * ldr;
            S.st_b = Rf + (int64_t)(2 * t + 1) * ldr;
        }
        UOT_HIP(launch_adj(p->k_dtype, B.nc, ADJ_STEP, (int)dim, S, stream), "adjoint step pass");
        if (t > 1) {
            AdjColLaunch C3 = Cc;
            C3.partials = A.partials;
            C3.G = B.G;
            C3.acc64 = (p->k_dtype == UOT_F64);
            C3.mode = ADJ_COL_STEP;
            C3.v = vprev;
            C3.w = (double*)wprev;
            UOT_HIP(launch_adj_col(C3, stream), "adjoint columns");
        }
        return UOT_OK;
    };
    if (B.stored) {
        const double* tv = ckpt;                       // v_0 .. v_T
        const double* tw = tv + (size_t)(T + 1) * m;   // K^T u_1 .. K^T u_T
        const double* tu = tw + (size_t)T * m;         // u_1 .. u_T
        const double* ts = tu + (size_t)T * n;         // K v_0 .. K v_{T-1}
        for (int t = T; t >= 1; --t) {
            st = reverse_step(t, tv + (size_t)(t - 1) * m, tu + (size_t)(t - 1) * n, ts + (size_t)(t - 1) * n,
                              t > 1 ? tw + (size_t)(t - 2) * m : nullptr);
            if (st != UOT_OK) return st;
        }
    }
    for (int c = B.nseg - 1; c >= 0; --c) {
        const int t0 = c * B.k;
        const int len = std::min(B.k, T - t0);
        const double* v0 = ckpt + (size_t)c * 2 * m;
        const double* w0 = v0 + m;
        for (int q = 0; q < len; ++q) {
            PassLaunch LF = L;
            LF.v = (q == 0) ? v0 : vtr + (size_t)(q - 1) * m;
            LF.u = utr + (size_t)q * n;
            LF.s_trace = str + (size_t)q * n;
            UOT_HIP(launch_pass(P.k_dtype, P.acc64, MODE_FUSED, P.shape, LF, stream), "recompute pass");
            FinLaunch FF = F;
            FF.v = vtr + (size_t)q * m;
            FF.w_out = wtr + (size_t)q * m;
            UOT_HIP(launch_finalize(FF, stream), "recompute finalize");
        }
        for (int q = len - 1; q >= 0; --q) {
            st = reverse_step(t0 + q + 1, (q == 0) ? v0 : vtr + (size_t)(q - 1) * m, utr + (size_t)q * n,
                              str + (size_t)q * n, (q == 0) ? w0 : wtr + (size_t)(q - 1) * m);
            if (st != UOT_OK) return st;
        }
    }
    AdjFinish Fin;
    memset(&Fin, 0, sizeof(Fin));
    Fin.grad_loss = grad_loss;
    Fin.abar = abar;
    Fin.bbar = bbar;
    Fin.gsum = gsum;
    Fin.gy = gy;
    Fin.x = x;
    Fin.grad_a = grad_a;
    Fin.grad_b = grad_b;
    Fin.grad_x = grad_x;
    Fin.n = n;
    Fin.m = m;
    Fin.dim = (int32_t)dim;
    UOT_HIP(launch_adj_finish(Fin, stream), "adjoint finish");
    if (cost_grad) {
        GradCLaunch G;
        memset(&G, 0, sizeof(G));
        G.K = K;
        G.k_dtype = p->k_dtype;
        G.ldk = ldk;
        G.n = n;
        G.m = m;
        G.nterms = B.nterms;
        G.Lf = Lf;
        G.Rf = Rf;
        G.ldl = ldl;
        G.ldr = ldr;
        G.grad_loss = grad_loss;
        G.inv_eps = 1.0 / p->eps;
        G.G = grad_C;
        G.ldg = ldgc;
        G.x = x;
        G.dim = (int32_t)dim;
        G.ysum = grad_y ? (double*)(base + B.off_ysum) : nullptr;
        UOT_HIP(launch_gradc(G, stream), "cost gradient product");
        if (grad_y)
            UOT_HIP(launch_grady_finish(G.ysum, B.row_tiles, y, m, (int32_t)dim, grad_y, stream), "target gradient");
    }
    return UOT_OK;
}


// ---------------------------------------------------------------------------
// The paper's literal in-place matrix rescaling
// ---------------------------------------------------------------------------
uot_status make_matrix_plan(const uot_problem* p, const uot_options* o, Plan& P) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (!p->K) return fail(UOT_ERR_ARG, "the in-place form rescales the matrix given as K");
    if (p->k_dtype != UOT_F32 && p->k_dtype != UOT_F64)
        return fail(UOT_ERR_DTYPE, "the in-place form rescales an FP32 or FP64 matrix");
    if (o->absorb_log_threshold != 0.0 || records_iterates(o) || o->persistent || o->u0 || o->v0 || !o->fused ||
        (p->k_dtype == UOT_F32 && o->accum == UOT_ACC_F64))
        return fail(UOT_ERR_UNSUPPORTED,
                    "the in-place form runs the fused per-iteration pass with the storage type's own arithmetic: "
                    "no absorption, checkpoints, warm start, cooperative loop or FP64 accumulation of FP32");
    if (o->tune > 8) return fail(UOT_ERR_UNSUPPORTED, "the in-place form runs the one-row launch shapes (tune 1-8)");
    if (p->k_scale != 0.0 && p->k_scale != 1.0) return fail(UOT_ERR_ARG, "the in-place form takes k_scale 1");
    return make_plan(p, o, P, true);
}

uot_status run_matrix(const uot_problem* p, const uot_options* o, const uot_outputs* out, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
    Plan P;
    uot_status st = make_matrix_plan(p, o, P);
    if (st != UOT_OK) return st;
    if (!out || !out->u || !out->v) return fail(UOT_ERR_ARG, "outputs u and v are required");
    if (!aligned(out->u, 8) || !aligned(out->v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if (ws_bytes < P.total || !ws) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    PinnedGuard pin;
    if (o->tol > 0.0) UOT_HIP(pinned_acquire(pin.slot), "hipHostMalloc");
    uint32_t* flag_host = o->tol > 0.0 ? pin.slot.flag() : nullptr;
    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* cprev = (double*)(base + P.off_cprev);
    double* wbuf = (double*)(base + P.off_w);
    double* bp = (double*)(base + P.off_bp);
    void* part = base + P.off_part;
    double* alpha = out->u;      // row factors of the last iteration (1 before the first)
    double* beta = out->v;       // column factors the next iteration applies
    // u = 1 (it weights the first column sums), beta = 1 (so the first factors are (b / colsum)^fi)
    UOT_HIP(launch_init(alpha, p->n, nullptr, beta, p->m, nullptr, cprev, ctrl, stream), "init");
    const double fi = fi_of(p->eps, p->tau);

    PassLaunch L;
    memset(&L, 0, sizeof(L));
    L.K = p->K;
    L.ldk = p->ldk;
    L.n = p->n;
    L.m = p->m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.v = beta;
    L.a = p->a;
    L.u = alpha;
    L.s_out = out->r;
    L.partials = part;
    L.ldp = P.ldp;
    L.fi = fi;
    L.fi_is_one = (fi == 1.0);
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.check_done = 1;
    L.ldv_bytes = P.ldv_bytes;
    L.k_scale = 1.0;
    L.tol = o->tol;
    L.fin_blocks = P.fin_blocks;
    L.blockpart = bp;
    FinLaunch F;
    memset(&F, 0, sizeof(F));
    F.partials = part;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = p->m;
    F.b = p->b;
    F.v = beta;
    F.w_out = wbuf;
    F.cprev = cprev;
    F.k_scale = 1.0;
    F.fi = fi;
    F.fi_is_one = (fi == 1.0);
    F.inv_eps = 1.0 / p->eps;
    F.ctrl = ctrl;
    F.blockpart = bp;
    F.acc64 = P.acc64;

    // Before the first iteration: column sums of A (rows weighted by u = 1),
    // then the first column factors.
    {
        PassLaunch LC = L;
        LC.check_done = 0;
        UOT_HIP(launch_pass(P.k_dtype, P.acc64, MODE_COL, P.shape, LC, stream), "column sums");
        UOT_HIP(launch_finalize(F, stream), "column factors");
    }
    const int check_every = o->check_every > 0 ? o->check_every : 1;
    int64_t iters_run = 0;
    for (int t = 0; t < o->max_iter; ++t) {
        PassLaunch L1 = L;
        L1.iter = t + 1;
        L1.test_stop = 1;
        UOT_HIP(launch_pass_matrix(P.k_dtype, P.shape, L1, stream), "in-place pass");
        UOT_HIP(launch_finalize(F, stream), "column factors");
        iters_run = t + 1;
        if (flag_host && (t + 1) % check_every == 0 && t + 1 < o->max_iter) {
            UOT_HIP(hipMemcpyAsync(flag_host, &ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                    "flag copy");
            UOT_HIP(hipStreamSynchronize(stream), "flag sync");
            if (*(volatile uint32_t*)flag_host) break;
        }
    }
    if (out->c && o->max_iter > 0)
        UOT_HIP(hipMemcpyAsync(out->c, wbuf, sizeof(double) * p->m, hipMemcpyDeviceToDevice, stream), "column sums");
    if (out->info) {
        ObjLaunch O;
        memset(&O, 0, sizeof(O));
        O.n = p->n;
        O.m = p->m;
        O.eps = p->eps;
        O.info = out->info;
        O.ctrl = ctrl;
        O.tol = o->tol;
        O.iters_run = iters_run;
        O.blockpart = bp;
        O.fin_blocks = P.fin_blocks;
        O.info_only = 1;
        UOT_HIP(launch_objective(O, stream), "report");
    }
    return UOT_OK;
}

// ---------------------------------------------------------------------------
// Kernel-free solve from points (the Gibbs kernel recomputed in every pass)
// ---------------------------------------------------------------------------
// Widest rows of the kernel-free solve (the column-tiled form's row-sum
// buffer holds ceil(m / 8192) doubles per row).
constexpr int64_t kPointsMaxM = 1 << 20;

struct PtsPlan {
    int32_t G;
    int64_t rows_per_wg, ldp;
    int32_t fin_blocks;
    int32_t tiles;        // 0: fused pass; > 0: column-tiled row and column passes
    size_t off_ctrl, off_cprev, off_w, off_s, off_bp, off_part, off_rows, off_beta, off_loga, off_rowpart, total;
};

uot_status make_points_plan(const uot_problem* p, int64_t dim, double cost_scale, const uot_options* o,
                            PtsPlan& P) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "empty problem (n=%lld, m=%lld)", (long long)p->n, (long long)p->m);
    if (!p->a || !p->b) return fail(UOT_ERR_ARG, "a and b must not be NULL");
    if (!aligned(p->a, 8) || !aligned(p->b, 8)) return fail(UOT_ERR_ALIGN, "a and b must be 8-byte aligned");
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "tau must be > 0 (or +inf)");
    if (!(cost_scale > 0.0) || !isfinite(cost_scale)) return fail(UOT_ERR_ARG, "cost_scale must be finite and > 0");
    if (dim != 2 && dim != 3) return fail(UOT_ERR_UNSUPPORTED, "point dimension %lld (2 or 3)", (long long)dim);
    if (p->m > kPointsMaxM)
        return fail(UOT_ERR_UNSUPPORTED, "the kernel-free solve takes rows of up to %lld columns (m=%lld)",
                    (long long)kPointsMaxM, (long long)p->m);
    if (o->max_iter < 0) return fail(UOT_ERR_ARG, "max_iter must be >= 0");
    if (o->absorb_log_threshold != 0.0 || records_iterates(o) || o->persistent || !o->fused ||
        o->accum != UOT_ACC_F32)
        return fail(UOT_ERR_UNSUPPORTED,
                    "the kernel-free solve runs the fused per-iteration pass with FP32 lane arithmetic: no "
                    "absorption, checkpoints, cooperative loop or FP64 accumulation");
    if (o->u0 && !aligned(o->u0, 8)) return fail(UOT_ERR_ALIGN, "u0 must be 8-byte aligned");
    if (o->v0 && !aligned(o->v0, 8)) return fail(UOT_ERR_ALIGN, "v0 must be 8-byte aligned");
    // As many workgroups as the compute units hold at once (the pass is
    // ALU-bound: one wave of strips, no tail), each with at least one full
    // group of rows.  Rows wider than the fused pass holds run as strips x
    // column tiles.
    P.tiles = p->m > online_max_m() ? (int32_t)((p->m + online_tile_cols() - 1) / online_tile_cols()) : 0;
    if (P.tiles > 0) {
        const int per_cu = std::max(1, online_tile_wgs_per_cu((int)dim));
        const int64_t strips = std::max<int64_t>(1, (int64_t)per_cu * cu_count() / P.tiles);
        const int64_t target = std::min<int64_t>(strips, (p->n + 7) / 8);
        P.rows_per_wg = (p->n + target - 1) / target;
    } else {
        const int per_cu = std::max(1, online_wgs_per_cu((int)dim, p->m));
        const int64_t rg = std::max(1, online_rows_per_group((int)dim, p->m));
        const int64_t target = std::min<int64_t>((int64_t)per_cu * cu_count(), (p->n + rg - 1) / rg);
        P.rows_per_wg = (p->n + target - 1) / target;
    }
    P.G = (int32_t)((p->n + P.rows_per_wg - 1) / P.rows_per_wg);
    P.ldp = round_up(p->m, 64);
    P.fin_blocks = finalize_blocks(p->m);
    size_t off = 0;
    P.off_ctrl = off; off = align_up(off + sizeof(Ctrl), kAlign);
    P.off_cprev = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_w = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_s = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.off_bp = off; off = align_up(off + sizeof(double) * 2 * (size_t)P.fin_blocks, kAlign);
    P.off_part = off; off = align_up(off + sizeof(float) * (size_t)P.G * P.ldp, kAlign);
    P.off_rows = off; off = align_up(off + sizeof(double) * 4 * (size_t)p->n, kAlign);
    P.off_beta = off; off = align_up(off + sizeof(double) * (size_t)p->m, kAlign);
    P.off_loga = off; off = align_up(off + sizeof(double) * (size_t)p->n, kAlign);
    P.off_rowpart = off; off = align_up(off + sizeof(double) * (size_t)P.tiles * p->n, kAlign);
    P.total = off;
    return UOT_OK;
}

uot_status run_points(const uot_problem* p, const double* x, const double* y, int64_t dim, double cost_scale,
                      const uot_options* o, const uot_outputs* out, void* ws, size_t ws_bytes, hipStream_t stream) {
    PtsPlan P;
    uot_status st = make_points_plan(p, dim, cost_scale, o, P);
    if (st != UOT_OK) return st;
    if (!x || !y) return fail(UOT_ERR_ARG, "x and y must not be NULL");
    if (!aligned(x, 8) || !aligned(y, 8)) return fail(UOT_ERR_ALIGN, "x and y must be 8-byte aligned");
    if (!out || !out->u || !out->v) return fail(UOT_ERR_ARG, "outputs u and v are required");
    if (!aligned(out->u, 8) || !aligned(out->v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if (ws_bytes < P.total || !ws) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    PinnedGuard pin;
    if (o->tol > 0.0) UOT_HIP(pinned_acquire(pin.slot), "hipHostMalloc");
    uint32_t* flag_host = o->tol > 0.0 ? pin.slot.flag() : nullptr;
    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* cprev = (double*)(base + P.off_cprev);
    double* wbuf = (double*)(base + P.off_w);
    double* sbuf = (double*)(base + P.off_s);
    double* bp = (double*)(base + P.off_bp);
    void* part = base + P.off_part;
    const double fi = fi_of(p->eps, p->tau);
    double* rows = (double*)(base + P.off_rows);
    double* beta = (double*)(base + P.off_beta);
    double* loga = (double*)(base + P.off_loga);
    const double c2 = cost_scale * 1.4426950408889634 / p->eps;      // log2(e) / eps
    UOT_HIP(launch_init(out->u, p->n, o->u0, out->v, p->m, o->v0, cprev, ctrl, stream), "init");
    UOT_HIP(launch_online_setup(x, y, p->a, p->n, p->m, (int)dim, c2, rows, beta, loga, stream), "point terms");

    OnlineLaunch OL;
    memset(&OL, 0, sizeof(OL));
    PassLaunch& L = OL.P;
    L.n = p->n;
    L.m = p->m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.v = out->v;
    L.a = p->a;
    L.u = out->u;
    L.partials = part;
    L.ldp = P.ldp;
    L.fi = fi;
    L.fi_is_one = (fi == 1.0);
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.check_done = 1;
    L.tol = o->tol;
    L.fin_blocks = P.fin_blocks;
    L.blockpart = bp;
    L.k_scale = 1.0;
    OL.y = y;
    OL.rows = rows;
    OL.beta = beta;
    OL.loga = loga;
    OL.dim = (int32_t)dim;
    OL.rowpart = (double*)(base + P.off_rowpart);
    OL.tiles = P.tiles;

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
    F.k_scale = 1.0;
    F.fi = fi;
    F.fi_is_one = (fi == 1.0);
    F.inv_eps = 1.0 / p->eps;
    F.ctrl = ctrl;
    F.blockpart = bp;
    F.acc64 = 0;

    const int check_every = o->check_every > 0 ? o->check_every : 1;
    int64_t iters_run = 0;
    for (int t = 0; t < o->max_iter; ++t) {
        OnlineLaunch O1 = OL;
        O1.P.iter = t + 1;
        O1.P.test_stop = 1;
        if (P.tiles > 0) {
            UOT_HIP(launch_online_tile_rows(O1, stream), "kernel-free row pass");
            UOT_HIP(launch_online_row_finish(OL, 0, stream), "row finish");
            UOT_HIP(launch_online_tile_cols(OL, stream), "kernel-free column pass");
        } else {
            UOT_HIP(launch_online(MODE_FUSED, O1, stream), "kernel-free pass");
        }
        UOT_HIP(launch_finalize(F, stream), "column finalize");
        iters_run = t + 1;
        if (flag_host && (t + 1) % check_every == 0 && t + 1 < o->max_iter) {
            UOT_HIP(hipMemcpyAsync(flag_host, &ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                    "flag copy");
            UOT_HIP(hipStreamSynchronize(stream), "flag sync");
            if (*(volatile uint32_t*)flag_host) break;
        }
    }
    // Marginals of the final scalings, then the objective.
    {
        OnlineLaunch OM = OL;
        OM.P.check_done = 0;
        OM.P.s_out = sbuf;
        if (P.tiles > 0) {
            UOT_HIP(launch_online_tile_rows(OM, stream), "kernel-free row pass");
            UOT_HIP(launch_online_row_finish(OM, 1, stream), "row sums");
            UOT_HIP(launch_online_tile_cols(OM, stream), "kernel-free column pass");
        } else {
            UOT_HIP(launch_online(MODE_MARG, OM, stream), "kernel-free marginal pass");
        }
        FinLaunch FM = F;
        FM.marginal_only = 1;
        FM.c_out = nullptr;
        UOT_HIP(launch_finalize(FM, stream), "marginal finalize");
    }
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
    O.f_out = out->f;
    O.g_out = out->g;
    O.blockpart = bp;
    O.fin_blocks = P.fin_blocks;
    UOT_HIP(launch_objective(O, stream), "objective");
    return UOT_OK;
}

// ---------------------------------------------------------------------------
// Log-domain (log-sum-exp) solve with an optional eps-scaling schedule
// ---------------------------------------------------------------------------
struct LsePlan {
    int32_t G;
    int64_t rows_per_wg, ldp, ldc32;
    int32_t fin_blocks;
    size_t off_ctrl, off_cprev, off_f, off_g, off_la2, off_lb2, off_ones_n, off_ones_m, off_r, off_c, off_bp,
        off_pmax, off_psum, off_c32, total;
};

uot_status make_lse_plan(const uot_problem* p, const uot_options* o, const uot_eps_schedule* sch, LsePlan& P) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "empty problem (n=%lld, m=%lld)", (long long)p->n, (long long)p->m);
    if (!p->a || !p->b) return fail(UOT_ERR_ARG, "a and b must not be NULL");
    if (!p->C) return fail(UOT_ERR_ARG, "the log-domain solve reads the cost C (NULL given)");
    if (!aligned(p->a, 8) || !aligned(p->b, 8)) return fail(UOT_ERR_ALIGN, "a and b must be 8-byte aligned");
    if (!aligned(p->C, 16) || p->ldc < p->m || p->ldc % 2 != 0)
        return fail(UOT_ERR_ALIGN, "C must be 16-byte aligned with an even ldc >= m");
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "tau must be > 0 (or +inf)");
    if (p->k_dtype != UOT_F64 && p->k_dtype != UOT_F32)
        return fail(UOT_ERR_DTYPE, "the cost is read as FP64 or FP32 (k_dtype %d)", (int)p->k_dtype);
    if (p->m > lse_max_m(p->k_dtype))
        return fail(UOT_ERR_UNSUPPORTED, "rows of at most %lld columns for this cost storage (m=%lld)",
                    (long long)lse_max_m(p->k_dtype), (long long)p->m);
    if (o->max_iter < 0) return fail(UOT_ERR_ARG, "max_iter must be >= 0");
    if (o->absorb_log_threshold != 0.0 || records_iterates(o) || o->persistent || !o->fused || o->u0 || o->v0 ||
        o->accum != UOT_ACC_F32)
        return fail(UOT_ERR_UNSUPPORTED,
                    "the log-domain solve runs its own fused pass: no absorption, checkpoints, cooperative loop, "
                    "warm start or accumulation option");
    if (sch) {
        if (sch->eps0 > p->eps) {
            if (!(sch->factor > 0.0 && sch->factor < 1.0)) return fail(UOT_ERR_ARG, "eps-scaling factor must lie in (0, 1)");
            if (sch->stage_iters < 1) return fail(UOT_ERR_ARG, "eps-scaling stages need stage_iters >= 1");
            if (!isfinite(sch->eps0)) return fail(UOT_ERR_ARG, "eps0 must be finite");
        }
    }
    // One wave of workgroups over the compute units.
    const int per_cu = std::max(1, lse_wgs_per_cu(p->k_dtype, p->m));
    const int64_t target = std::min<int64_t>((int64_t)per_cu * cu_count(), p->n);
    P.rows_per_wg = (p->n + target - 1) / target;
    P.G = (int32_t)((p->n + P.rows_per_wg - 1) / P.rows_per_wg);
    P.ldp = round_up(p->m, 64);
    P.ldc32 = round_up(p->m, 4);
    const int64_t csize = p->k_dtype == UOT_F32 ? 4 : 8;
    const int64_t ldc_read = p->k_dtype == UOT_F32 ? P.ldc32 : p->ldc;
    if ((P.rows_per_wg + 4) * ldc_read * csize >= (1LL << 31))
        return fail(UOT_ERR_UNSUPPORTED, "a strip of %lld rows exceeds 2 GiB", (long long)P.rows_per_wg);
    P.fin_blocks = lse_finalize_blocks(p->m);
    size_t off = 0;
    P.off_ctrl = off; off = align_up(off + sizeof(Ctrl), kAlign);
    P.off_cprev = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_f = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.off_g = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_la2 = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.off_lb2 = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_ones_n = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.off_ones_m = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_r = off; off = align_up(off + sizeof(double) * p->n, kAlign);
    P.off_c = off; off = align_up(off + sizeof(double) * p->m, kAlign);
    P.off_bp = off; off = align_up(off + sizeof(double) * 2 * (size_t)P.fin_blocks, kAlign);
    P.off_pmax = off; off = align_up(off + sizeof(double) * (size_t)P.G * P.ldp, kAlign);
    P.off_psum = off; off = align_up(off + sizeof(float) * (size_t)P.G * P.ldp, kAlign);
    P.off_c32 = off;
    if (p->k_dtype == UOT_F32) off = align_up(off + sizeof(float) * (size_t)p->n * P.ldc32, kAlign);
    P.total = off;
    return UOT_OK;
}

uot_status run_lse(const uot_problem* p, const uot_options* o, const uot_eps_schedule* sch, const uot_outputs* out,
                   void* ws, size_t ws_bytes, hipStream_t stream) {
    LsePlan P;
    uot_status st = make_lse_plan(p, o, sch, P);
    if (st != UOT_OK) return st;
    if (!out || !out->u || !out->v) return fail(UOT_ERR_ARG, "outputs u and v are required");
    if (!aligned(out->u, 8) || !aligned(out->v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if (ws_bytes < P.total || !ws) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    PinnedGuard pin;
    if (o->tol > 0.0) UOT_HIP(pinned_acquire(pin.slot), "hipHostMalloc");
    uint32_t* flag_host = o->tol > 0.0 ? pin.slot.flag() : nullptr;
    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* cprev = (double*)(base + P.off_cprev);
    double* f = (double*)(base + P.off_f);
    double* g = (double*)(base + P.off_g);
    double* la2 = (double*)(base + P.off_la2);
    double* lb2 = (double*)(base + P.off_lb2);
    double* ones_n = (double*)(base + P.off_ones_n);
    double* ones_m = (double*)(base + P.off_ones_m);
    double* rbuf = (double*)(base + P.off_r);
    double* cbuf = (double*)(base + P.off_c);
    double* bp = (double*)(base + P.off_bp);
    double* pmax = (double*)(base + P.off_pmax);
    float* psum = (float*)(base + P.off_psum);
    const void* Cread = p->C;
    int64_t ldc_read = p->ldc;
    if (p->k_dtype == UOT_F32) {
        float* c32 = (float*)(base + P.off_c32);
        UOT_HIP(launch_cost_to_f32(p->C, p->ldc, p->n, p->m, c32, P.ldc32, stream), "cost to FP32");
        Cread = c32;
        ldc_read = P.ldc32;
    }
    // init: u = v = 1 in the ones vectors, f = g = 0, flags and stop state cleared
    UOT_HIP(launch_init(ones_n, p->n, nullptr, ones_m, p->m, nullptr, cprev, ctrl, stream), "init");
    UOT_HIP(launch_fill_f64(f, p->n, 0.0, stream), "f");
    UOT_HIP(launch_fill_f64(g, p->m, 0.0, stream), "g");
    UOT_HIP(launch_lse_setup(p->a, p->n, p->b, p->m, la2, lb2, stream), "log targets");

    LseLaunch L;
    memset(&L, 0, sizeof(L));
    L.P.n = p->n;
    L.P.m = p->m;
    L.P.rows_per_wg = P.rows_per_wg;
    L.P.grid = P.G;
    L.P.ctrl = ctrl;
    L.P.check_done = 1;
    L.P.tol = o->tol;
    L.P.fin_blocks = P.fin_blocks;
    L.P.blockpart = bp;
    L.C = Cread;
    L.c_dtype = p->k_dtype;
    L.ldc = ldc_read;
    L.g = g;
    L.f = f;
    L.la2 = la2;
    L.pmax = pmax;
    L.psum = psum;
    L.ldp = P.ldp;
    LseFinLaunch F;
    memset(&F, 0, sizeof(F));
    F.pmax = pmax;
    F.psum = psum;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = p->m;
    F.lb2 = lb2;
    F.g = g;
    F.cprev = cprev;
    F.ctrl = ctrl;
    F.blockpart = bp;

    // Stages: eps0 factor^k down to eps (stage_iters each), then eps (max_iter, stopping rule).
    const bool scaled = sch && sch->eps0 > p->eps;
    double e = scaled ? sch->eps0 : p->eps;
    const int check_every = o->check_every > 0 ? o->check_every : 1;
    int64_t total = 0;
    for (;;) {
        const bool last = !(e > p->eps);
        const double fi = fi_of(e, p->tau);
        L.c = 1.4426950408889634 / e;
        L.inv_c = e * 0.6931471805599453;
        L.fi = fi;
        F.c = L.c;
        F.inv_c = L.inv_c;
        F.fi = fi;
        const int64_t T = last ? o->max_iter : sch->stage_iters;
        if (last && total > 0) UOT_HIP(launch_fill_f64(cprev, p->m, 0.0, stream), "stage reset");
        for (int64_t t = 0; t < T; ++t) {
            LseLaunch L1 = L;
            L1.P.iter = total + 1;
            L1.P.test_stop = (last && t > 0) ? 1 : 0;      // the stage's first iteration has no previous marginal
            UOT_HIP(launch_lse(MODE_FUSED, L1, stream), "log-domain pass");
            UOT_HIP(launch_lse_finalize(F, stream), "log-domain finalize");
            ++total;
            if (last && flag_host && (t + 1) % check_every == 0 && t + 1 < T) {
                UOT_HIP(hipMemcpyAsync(flag_host, &ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                        "flag copy");
                UOT_HIP(hipStreamSynchronize(stream), "flag sync");
                if (*(volatile uint32_t*)flag_host) break;
            }
        }
        if (last) break;
        e = e * sch->factor > p->eps ? e * sch->factor : p->eps;
    }
    // Marginals at the final potentials, then the objective in potential form.
    {
        LseLaunch LM = L;
        LM.P.check_done = 0;
        LM.P.test_stop = 0;
        LM.r_out = rbuf;
        UOT_HIP(launch_lse(MODE_MARG, LM, stream), "log-domain marginal pass");
        LseFinLaunch FM = F;
        FM.marginal_only = 1;
        FM.c_out = cbuf;
        UOT_HIP(launch_lse_finalize(FM, stream), "log-domain marginal finalize");
    }
    ObjLaunch O;
    memset(&O, 0, sizeof(O));
    O.u = ones_n;
    O.v = ones_m;
    O.s = rbuf;
    O.w = cbuf;
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
    O.iters_run = total;
    O.blockpart = bp;
    O.fin_blocks = P.fin_blocks;
    O.fpot = f;
    O.gpot = g;
    O.f_out = out->f;
    O.g_out = out->g;
    O.u_tot = out->u;
    O.v_tot = out->v;
    UOT_HIP(launch_objective(O, stream), "objective");
    return UOT_OK;
}

// ---------------------------------------------------------------------------
// Implicit (envelope) backward: marginal passes only
// ---------------------------------------------------------------------------
struct ImpPlan {
    Plan F;                   // forward plan (the marginal passes)
    size_t off_sy, off_wx, off_ud, off_vd, total;
};

uot_status make_imp_plan(const uot_problem* p, const uot_options* o, int64_t dim, ImpPlan& B) {
    if (!o) return fail(UOT_ERR_ARG, "options must not be NULL");
    uot_options fo = *o;
    fo.fused = 1;
    fo.persistent = 0;
    fo.tol = 0.0;
    fo.absorb_log_threshold = 0.0;
    fo.checkpoint_every = 0;
    fo.store_iterates = 0;
    fo.u0 = fo.v0 = nullptr;
    fo.max_iter = 1;
    uot_status st = make_plan(p, &fo, B.F);
    if (st != UOT_OK) return st;
    if (dim < 0 || dim > 16) return fail(UOT_ERR_UNSUPPORTED, "point dimension %lld (0 to 16)", (long long)dim);
    const size_t d8 = sizeof(double);
    size_t off = B.F.total;
    B.off_sy = off; off = align_up(off + d8 * (size_t)(dim > 0 ? dim : 1) * p->n, kAlign);
    B.off_wx = off; off = align_up(off + d8 * (size_t)(dim > 0 ? dim : 1) * p->m, kAlign);
    B.off_ud = off; off = align_up(off + d8 * (size_t)p->n, kAlign);
    B.off_vd = off; off = align_up(off + d8 * (size_t)p->m, kAlign);
    B.total = off;
    return UOT_OK;
}

uot_status run_implicit_backward(const uot_problem* p, const uot_options* o, const double* u, const double* v,
                                 const double* grad_loss, double* grad_a, double* grad_b, double* grad_C,
                                 int64_t ldgc, const double* x, const double* y, int64_t dim, double* grad_x,
                                 double* grad_y, void* ws, size_t ws_bytes, hipStream_t stream) {
    ImpPlan B;
    uot_status st = make_imp_plan(p, o, dim, B);
    if (st != UOT_OK) return st;
    if (!u || !v || !grad_loss) return fail(UOT_ERR_ARG, "u, v and grad_loss are required");
    if (!aligned(u, 8) || !aligned(v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
    if ((grad_x || grad_y) && (dim < 1 || !x || !y)) return fail(UOT_ERR_ARG, "point gradients need x, y and dim >= 1");
    if (grad_C && ldgc < p->m) return fail(UOT_ERR_ARG, "ldgc (%lld) < m (%lld)", (long long)ldgc, (long long)p->m);
    if ((grad_C && !aligned(grad_C, 8)) || (grad_x && !aligned(grad_x, 8)) || (grad_y && !aligned(grad_y, 8)))
        return fail(UOT_ERR_ALIGN, "gradient outputs must be 8-byte aligned");
    if (ws_bytes < B.total || !ws) return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", B.total, ws_bytes);
    if (!aligned(ws, kAlign)) return fail(UOT_ERR_ALIGN, "workspace must be 256-byte aligned");
    const Plan& P = B.F;
    const int64_t n = p->n, m = p->m;
    char* base = (char*)ws;
    Ctrl* ctrl = (Ctrl*)(base + P.off_ctrl);
    double* sbuf = (double*)(base + P.off_s);
    double* wbuf = (double*)(base + P.off_w);
    double* bp = (double*)(base + P.off_bp);
    void* part = base + P.off_part;
    double* sy = (double*)(base + B.off_sy);
    double* wx = (double*)(base + B.off_wx);
    double* ud = (double*)(base + B.off_ud);
    double* vd = (double*)(base + B.off_vd);
    const void* K = p->K;
    int64_t ldk = p->ldk;
    const double store_scale = (p->k_dtype == UOT_FP8_E4M3) ? 448.0 : 1.0;
    double k_scale = (p->K && p->k_scale > 0.0) ? p->k_scale : 1.0;
    if (P.build_k) {
        K = base + P.off_k;
        ldk = P.ldk_ws;
        k_scale = 1.0 / store_scale;
        UOT_HIP(launch_kernel_build(p->C, p->ldc, n, m, p->eps, nullptr, nullptr, p->k_dtype, (void*)K, ldk,
                                    store_scale, stream),
                "kernel build");
    }
    UOT_HIP(launch_init(nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, ctrl, stream), "init");

    PassLaunch L;
    memset(&L, 0, sizeof(L));
    L.K = K;
    L.ldk = ldk;
    L.n = n;
    L.m = m;
    L.rows_per_wg = P.rows_per_wg;
    L.grid = P.G;
    L.a = p->a;
    L.partials = part;
    L.ldp = P.ldp;
    L.fi = fi_of(p->eps, p->tau);
    L.fi_is_one = (L.fi == 1.0);
    L.inv_eps = 1.0 / p->eps;
    L.ctrl = ctrl;
    L.check_done = 0;
    L.ldv_bytes = P.ldv_bytes;
    L.k_scale = k_scale;
    L.fin_blocks = P.fin_blocks;
    L.blockpart = bp;
    FinLaunch F;
    memset(&F, 0, sizeof(F));
    F.partials = part;
    F.ldp = P.ldp;
    F.G = P.G;
    F.m = m;
    F.b = p->b;
    F.k_scale = k_scale;
    F.fi = L.fi;
    F.fi_is_one = L.fi_is_one;
    F.inv_eps = L.inv_eps;
    F.ctrl = ctrl;
    F.blockpart = bp;
    F.acc64 = P.acc64;
    F.marginal_only = 1;
    F.c_out = nullptr;

    // one marginal pass: s = K v (rows), w = K^T u (columns)
    auto marginals = [&](const double* uu, const double* vv, double* s_out, double* w_out) -> hipError_t {
        PassLaunch LM = L;
        LM.u = (double*)uu;
        LM.v = vv;
        LM.s_out = s_out;
        hipError_t e = launch_pass(P.k_dtype, P.acc64, MODE_MARG, P.shape, LM, stream);
        if (e != hipSuccess) return e;
        FinLaunch FM = F;
        FM.v = (double*)vv;   // read only (c_out is NULL)
        FM.w_out = w_out;
        return launch_finalize(FM, stream);
    };
    UOT_HIP(marginals(u, v, sbuf, wbuf), "marginal pass");
    const bool points = grad_x || grad_y;
    for (int d = 0; points && d < dim; ++d) {
        UOT_HIP(launch_env_weight(u, x, n, v, y, m, (int32_t)dim, d, ud, vd, stream), "point weights");
        UOT_HIP(marginals(ud, vd, sy + (int64_t)d * n, wx + (int64_t)d * m), "marginal pass");
    }
    EnvFinish E;
    memset(&E, 0, sizeof(E));
    E.grad_loss = grad_loss;
    E.u = u;
    E.v = v;
    E.a = p->a;
    E.b = p->b;
    E.s = sbuf;
    E.w = wbuf;
    E.sy = sy;
    E.wx = wx;
    E.x = x;
    E.y = y;
    E.grad_a = grad_a;
    E.grad_b = grad_b;
    E.grad_x = grad_x;
    E.grad_y = grad_y;
    E.n = n;
    E.m = m;
    E.dim = points ? (int32_t)dim : 0;
    E.tau_inf = isinf(p->tau) ? 1 : 0;
    E.tau = p->tau;
    UOT_HIP(launch_env_finish(E, stream), "envelope gradients");
    if (grad_C)
        UOT_HIP(launch_plan_from_k(K, p->k_dtype, ldk, n, m, k_scale, u, v, grad_C, UOT_F64, ldgc, stream, grad_loss),
                "cost gradient");
    return UOT_OK;
}

// ---------------------------------------------------------------------------
// Batched problems
// ---------------------------------------------------------------------------

uot_status check_batch_options(const uot_options* o) {
    if (!o) return fail(UOT_ERR_ARG, "options must not be NULL");
    if (o->max_iter < 0) return fail(UOT_ERR_ARG, "max_iter must be >= 0");
    if (o->tol > 0.0 && o->check_every < 1) return fail(UOT_ERR_ARG, "check_every must be >= 1");
    if (o->absorb_log_threshold != 0.0 || records_iterates(o) || o->persistent || o->u0 || o->v0)
        return fail(UOT_ERR_UNSUPPORTED,
                    "batched problems run the plain iteration: no absorption, checkpoints, warm start or "
                    "cooperative loop");
    return UOT_OK;
}

uot_status check_batch_problem(const uot_problem* p, const uot_outputs* out, int32_t idx) {
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "problem %d: empty (n=%lld, m=%lld)", idx, (long long)p->n, (long long)p->m);
    if (!p->a || !p->b) return fail(UOT_ERR_ARG, "problem %d: a and b must not be NULL", idx);
    if (!aligned(p->a, 8) || !aligned(p->b, 8)) return fail(UOT_ERR_ALIGN, "problem %d: a, b must be 8-byte aligned", idx);
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "problem %d: eps must be finite and > 0", idx);
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "problem %d: tau must be > 0 (or +inf)", idx);
    const int es = elem_size(p->k_dtype);
    if (es == 0) return fail(UOT_ERR_DTYPE, "problem %d: K dtype %d not supported", idx, (int)p->k_dtype);
    if (!p->K) return fail(UOT_ERR_ARG, "problem %d: batched problems take K (build it with uot_kernel_from_cost)", idx);
    if (p->ldk < p->m) return fail(UOT_ERR_ARG, "problem %d: ldk (%lld) < m (%lld)", idx, (long long)p->ldk, (long long)p->m);
    if (!aligned(p->K, 16) || p->ldk % (16 / es) != 0)
        return fail(UOT_ERR_ALIGN, "problem %d: K must be 16-byte aligned with ldk a multiple of %d", idx, 16 / es);
    if (p->n * p->ldk * es >= (int64_t)1 << 31)
        return fail(UOT_ERR_UNSUPPORTED, "problem %d: K of a batched problem must be below 2 GiB", idx);
    if (!(p->k_scale >= 0.0) || !isfinite(p->k_scale)) return fail(UOT_ERR_ARG, "problem %d: k_scale must be finite and >= 0", idx);
    if (!out) return fail(UOT_ERR_ARG, "outputs must not be NULL");
    if (!out->u || !out->v || !out->r || !out->c || !out->loss || !out->info)
        return fail(UOT_ERR_ARG, "problem %d: outputs u, v, r, c, loss and info are required", idx);
    if (!aligned(out->u, 8) || !aligned(out->v, 8) || !aligned(out->r, 8) || !aligned(out->c, 8) ||
        !aligned(out->loss, 8) || !aligned(out->info, 8))
        return fail(UOT_ERR_ALIGN, "problem %d: outputs must be 8-byte aligned", idx);
    return UOT_OK;
}

// Default tile shape: the smallest row-group capacity that covers m (lanes
// per row group x chunks), preferring more row groups (fewer barriers).
int batch_default_shape(int64_t m, int k_dtype) {
    int best = -1;
    int64_t best_cap = 0;
    for (int s = 0; s < batch_shape_count(); ++s) {
        if (!batch_shape_ok(s, k_dtype)) continue;
        const int64_t cap = batch_shape_max_m(s, k_dtype);
        if (cap < m) continue;
        if (best < 0 || cap < best_cap || (cap == best_cap && batch_shape_rows(s) > batch_shape_rows(best))) {
            best = s;
            best_cap = cap;
        }
    }
    return best;
}

int size_bucket(int64_t m) {
    int b = 0;
    while (((int64_t)1 << b) < m) ++b;
    return b;
}

// Autotuned shapes per (K dtype, column-count bucket), filled by timing runs.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tuned;

int batch_shape_for(int64_t m, int k_dtype) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find({k_dtype, size_bucket(m)});
        if (it != g_tuned.end() && batch_shape_max_m(it->second, k_dtype) >= m) return it->second;
    }
    return batch_default_shape(m, k_dtype);
}

// Splitting of large batched problems across workgroups (see pack_batch).
constexpr int kMaxParts = 4;            // parts per split problem
constexpr int32_t kMaxSplit = 256;      // split problems per batch
constexpr int64_t kMaxBatchM = 4096;    // widest batched row (FP8; FP32 and BF16 hold 2048)

int32_t batch_max_splits(int32_t count) { return std::min(count, kMaxSplit); }
// Queue entries: every problem, plus up to kMaxParts - 1 more per split problem.
int32_t batch_max_items(int32_t count) { return count + (kMaxParts - 1) * batch_max_splits(count); }
size_t batch_desc_bytes(int32_t count) {
    return align_up(sizeof(BatchDesc) * (size_t)std::max(batch_max_items(count), 1), kAlign);
}
size_t batch_pool_bytes(int32_t count) {
    const int32_t s = batch_max_splits(count);
    return align_up(kBatchHeaderBytes * (size_t)s, kAlign) + (size_t)s * align_up(batch_xch_bytes(kMaxParts, kMaxBatchM), kAlign);
}

// Queue entries of a batch.  A workgroup's time on a problem grows with the
// rows each of its row groups steps through, ceil(n / rg) per iteration,
// and with the chunks per lane (measured on the batched workload: about
// 0.7 us per row step at one chunk, 1.05 us at two, per iteration), so the
// estimated cost ceil(n / rg) (3 + nc) orders the queue, longest first.
// With `allow_split` (and a device to count the resident workgroups), a
// problem whose cost exceeds the average cost per workgroup is split by
// rows into up to kMaxParts parts that run on as many workgroups and
// exchange their column sums once per iteration.  Split problems go first
// in the queue, each with its parts consecutive, and all their parts
// together take at most 3/4 of the resident workgroups, so every part is
// running while its siblings wait for it.
struct BatchPack {
    std::vector<BatchDesc> d;
    int64_t m_lds = 0;
    int32_t nsplit = 0;
    size_t pool_used = 0;
};

int batch_grid_estimate(int k_dtype, int64_t m_cap);

uot_status pack_batch(const uot_problem* probs, int32_t count, const uot_options* o, const uot_outputs* outs,
                      bool allow_split, BatchPack& pk) {
    uot_status st = check_batch_options(o);
    if (st != UOT_OK) return st;
    if (count < 0) return fail(UOT_ERR_ARG, "count must be >= 0");
    if (count > 0 && (!probs || !outs)) return fail(UOT_ERR_ARG, "probs and outs must not be NULL");
    std::vector<int32_t> order(count);
    for (int32_t i = 0; i < count; ++i) {
        st = check_batch_problem(&probs[i], &outs[i], i);
        if (st != UOT_OK) return st;
        order[i] = i;
    }
    const int kd = count > 0 ? probs[0].k_dtype : UOT_F32;
    std::vector<int64_t> cost(count);
    for (int32_t i = 0; i < count; ++i) {
        const int sh = batch_shape_for(probs[i].m, kd);
        const int rg = sh >= 0 ? batch_shape_rows(sh) : 1;
        const int nc = sh >= 0 ? batch_shape_chunks(sh) : 1;
        cost[i] = (probs[i].n + rg - 1) / rg * (3 + nc);
    }
    auto work = [&](int32_t i) { return cost[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work(x) > work(y); });

    // parts per problem (in queue order)
    std::vector<int> parts(count, 1);
    int grid = 0;
    if (allow_split && count > 1) {
        int64_t m_cap = 0;
        for (int32_t i = 0; i < count; ++i) {
            const int sh = batch_shape_for(probs[i].m, kd);
            if (sh >= 0) m_cap = std::max(m_cap, batch_shape_max_m(sh, kd));
        }
        grid = batch_grid_estimate(kd, m_cap);
    }
    if (grid > 0 && count > 1) {
        int64_t total = 0;
        for (int32_t i = 0; i < count; ++i) total += work(i);
        const int64_t avg = std::max<int64_t>(1, total / grid);
        int budget = grid * 3 / 4;                   // workgroups the split parts may hold
        int32_t nsplit = 0;
        for (int32_t q = 0; q < count && nsplit < kMaxSplit; ++q) {
            const uot_problem& p = probs[order[q]];
            int pp = (int)std::min<int64_t>(kMaxParts, (work(order[q]) + avg - 1) / avg);
            pp = (int)std::min<int64_t>(pp, p.n / 16);
            // a part's time per iteration must stay well above the exchange's
            // few microseconds: at least 512 cost units (about 100 us) each
            pp = (int)std::min<int64_t>(pp, work(order[q]) / 512);
            if (pp < 2 || p.m > kMaxBatchM || pp > budget) break;
            parts[q] = pp;
            budget -= pp;
            ++nsplit;
        }
    }

    pk.d.clear();
    pk.m_lds = 0;
    pk.nsplit = 0;
    const int32_t nsplit_all = (int32_t)std::count_if(parts.begin(), parts.end(), [](int x) { return x > 1; });
    size_t xoff = align_up(kBatchHeaderBytes * (size_t)nsplit_all, kAlign);
    for (int32_t q = 0; q < count; ++q) {
        const uot_problem& p = probs[order[q]];
        const uot_outputs& out = outs[order[q]];
        if (p.k_dtype != kd) return fail(UOT_ERR_DTYPE, "all batched problems must share one K dtype");
        const int shape = batch_shape_for(p.m, kd);
        if (shape < 0)
            return fail(UOT_ERR_UNSUPPORTED, "problem %d: m = %lld exceeds the batched row capacity (%lld)",
                        order[q], (long long)p.m, (long long)batch_shape_max_m(batch_shape_count() - 1, kd));
        BatchDesc b{};
        b.K = p.K;
        b.ldk = p.ldk;
        b.n = p.n;
        b.m = p.m;
        b.a = p.a;
        b.b = p.b;
        b.u = (double*)out.u;
        b.v = (double*)out.v;
        b.r = out.r;
        b.c = out.c;
        b.loss = out.loss;
        b.info = out.info;
        b.fi = fi_of(p.eps, p.tau);
        b.fi_is_one = isinf(p.tau) ? 1 : 0;
        b.k_scale = p.k_scale > 0.0 ? p.k_scale : 1.0;
        b.eps = p.eps;
        b.tau = p.tau;
        b.shape = shape;
        b.index = order[q];
        b.part = 0;
        b.parts = 1;
        pk.m_lds = std::max(pk.m_lds, batch_shape_max_m(shape, kd));
        if (parts[q] == 1) {
            pk.d.push_back(b);
            continue;
        }
        const int P = parts[q];
        b.parts = P;
        b.split = pk.nsplit++;
        b.xch = (int64_t)xoff;
        xoff += align_up(batch_xch_bytes(P, p.m), kAlign);
        const int64_t rows = (p.n + P - 1) / P;
        const int es = elem_size(kd);
        for (int k = 0; k < P; ++k) {
            BatchDesc c = b;
            const int64_t r0 = k * rows;
            c.part = k;
            c.n = std::min(rows, p.n - r0);
            c.K = (const char*)p.K + r0 * p.ldk * es;
            c.a = (const double*)p.a + r0;
            c.u = (double*)out.u + r0;
            c.r = out.r + r0;
            pk.d.push_back(c);
        }
    }
    pk.pool_used = xoff;
    return UOT_OK;
}

// Resident workgroups of the batched kernel for a batch's LDS need (0
// without a device).
int batch_grid_estimate(int k_dtype, int64_t m_cap) {
    const size_t lds = batch_lds_bytes(m_cap);
    if ((int64_t)lds > max_lds_bytes()) return 0;
    return std::max(0, batch_max_grid(k_dtype, lds));
}

struct BatchRun {
    int k_dtype;
    int grid;
    size_t lds;
};

uot_status batch_launch_config(int k_dtype, int64_t m_lds, int32_t count, BatchRun& R) {
    R.k_dtype = k_dtype;
    R.lds = batch_lds_bytes(m_lds);
    if ((int64_t)R.lds > max_lds_bytes()) return fail(UOT_ERR_UNSUPPORTED, "batched LDS need exceeds the device");
    const int g = batch_max_grid(k_dtype, R.lds);
    if (g <= 0) return fail(UOT_ERR_HIP, "occupancy query failed for the batched kernel");
    R.grid = std::max(1, std::min(g, count));
    return UOT_OK;
}

// items: queue entries; nsplit, pool_bytes: the split problems and the bytes
// of exchange pool they use.  Workspace: the queue head, then (from
// kAlign + pool_offset) the exchange pool.
uot_status run_batch_packed(const BatchDesc* desc_dev, int32_t items, int32_t nsplit, size_t pool_offset,
                            size_t pool_bytes, int k_dtype, int64_t m_lds, const uot_options* o, void* ws,
                            size_t ws_bytes, uint64_t* trace, hipStream_t stream) {
    if (items == 0) return UOT_OK;
    if (!ws || ws_bytes < kAlign + pool_offset + pool_bytes || !aligned(ws, kAlign))
        return fail(UOT_ERR_WORKSPACE, "workspace too small or misaligned");
    BatchRun R;
    uot_status st = batch_launch_config(k_dtype, m_lds, items, R);
    if (st != UOT_OK) return st;
    BatchLaunch B;
    memset(&B, 0, sizeof(B));
    B.desc = desc_dev;
    B.count = items;
    B.max_iter = o->max_iter;
    B.tol = o->tol;
    B.check_every = std::max(o->check_every, 1);
    B.m_lds = m_lds;
    B.next = (uint32_t*)ws;
    B.trace = trace;
    B.pool = (unsigned char*)ws + kAlign + pool_offset;
    B.nsplit = nsplit;
    UOT_HIP(launch_batch(k_dtype, B, R.grid, R.lds, stream), "batched launch");
    return UOT_OK;
}

// Timing runs that pick the tile shape of each column-count bucket present
// in the batch (a few iterations of up to 8 of its problems per candidate).
uot_status autotune_batch(const uot_problem* probs, int32_t count, const uot_options* o, const uot_outputs* outs,
                          void* ws, size_t ws_bytes, hipStream_t stream) {
    const int kd = probs[0].k_dtype;
    std::map<int, std::vector<int32_t>> buckets;
    for (int32_t i = 0; i < count; ++i) buckets[size_bucket(probs[i].m)].push_back(i);
    const size_t dbytes = batch_desc_bytes(8);
    if (ws_bytes < kAlign + dbytes) return fail(UOT_ERR_WORKSPACE, "workspace too small for tuning");
    BatchDesc* ddev = (BatchDesc*)((char*)ws + kAlign);
    hipEvent_t e0, e1;
    UOT_HIP(hipEventCreate(&e0), "hipEventCreate");
    UOT_HIP(hipEventCreate(&e1), "hipEventCreate");
    uot_options t = *o;
    t.max_iter = std::min(o->max_iter, 3);
    t.tol = 0.0;
    uot_status st = UOT_OK;
    for (auto& kv : buckets) {
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            if (g_tuned.count({kd, kv.first})) continue;
        }
        std::vector<int32_t>& ids = kv.second;
        if (ids.size() > 8) ids.resize(8);
        int64_t mmax = 0;
        for (int32_t i : ids) mmax = std::max(mmax, probs[i].m);
        int best = -1;
        float best_ms = 0.0f;
        for (int s = 0; s < batch_shape_count() && st == UOT_OK; ++s) {
            if (!batch_shape_ok(s, kd) || batch_shape_max_m(s, kd) < mmax) continue;
            BatchPack pk;
            std::vector<uot_problem> ps;
            std::vector<uot_outputs> os;
            for (int32_t i : ids) {
                ps.push_back(probs[i]);
                os.push_back(outs[i]);
            }
            st = pack_batch(ps.data(), (int32_t)ps.size(), &t, os.data(), false, pk);      // no splitting
            if (st != UOT_OK) break;
            std::vector<BatchDesc>& d = pk.d;
            for (auto& b : d) b.shape = s;
            const int64_t m_lds = batch_shape_max_m(s, kd);
            hipError_t e = hipMemcpy(ddev, d.data(), sizeof(BatchDesc) * d.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) { st = hip_fail(e, "tuning copy"); break; }
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && st == UOT_OK; ++rep) {       // first run warms up
                e = hipEventRecord(e0, stream);
                if (e == hipSuccess)
                    st = run_batch_packed(ddev, (int32_t)d.size(), 0, dbytes, 0, kd, m_lds, &t, ws, ws_bytes, nullptr,
                                          stream);
                if (st == UOT_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
                if (st == UOT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
                if (st == UOT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess && st == UOT_OK) st = hip_fail(e, "tuning run");
            }
            if (st != UOT_OK) break;
            if (best < 0 || ms < best_ms) {
                best = s;
                best_ms = ms;
            }
        }
        if (st != UOT_OK) break;
        if (best >= 0) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[{kd, kv.first}] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}


// ---------------------------------------------------------------------------
// Many right-hand sides sharing one K
// ---------------------------------------------------------------------------

struct MultiGemmShape {
    int64_t rows_pad, kdim_pad, kchunk;
    int32_t splits;
};

// Split of the reduction: enough workgroups to fill the device (one per CU
// for the 256 x 256 tiles, which hold 120 KiB of LDS; about 512 for the
// 128 x 128 BF16 tiles, whose partial sums cost relatively more, 1024 for
// FP32; measured at 8192^2 x 256) with chunks of at least 256.  Rows are
// padded to the large tile whatever the variant.
MultiGemmShape multi_gemm_shape(int64_t rows, int64_t kdim_pad, int64_t r_pad, bool bf16, int variant) {
    MultiGemmShape g;
    g.rows_pad = round_up(rows, kMBigRows);
    g.kdim_pad = kdim_pad;
    const bool big = variant == 3;
    const int64_t tiles = big ? (r_pad / kMBigCols) * (g.rows_pad / kMBigRows)
                              : (r_pad / kMTileCols) * (g.rows_pad / kMTileRows);
    const int64_t target = big ? 256 : bf16 ? 512 : 1024;
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>(kdim_pad / 256, (target + tiles - 1) / tiles));
    g.kchunk = round_up((kdim_pad + splits - 1) / splits, 64);     // whole stages of every product variant
    g.splits = (int32_t)((kdim_pad + g.kchunk - 1) / g.kchunk);
    return g;
}

struct MultiPlan {
    bool bf16;
    int es;
    int variant;     // product kernel (MGemm::variant)
    bool blocked;    // K and K^T repacked into the tiled layout
    int64_t n, m, R, r_pad, ldn, ldm;
    MultiGemmShape row, col;
    size_t off_kt, off_kb, off_part, off_uhi, off_ulo, off_vhi, off_vlo, off_rm, off_cm, off_flags, total;
};

uot_status make_multi_plan(const uot_problem* p, int32_t R, const uot_options* o, MultiPlan& M) {
    if (!p || !o) return fail(UOT_ERR_ARG, "problem and options must not be NULL");
    if (p->n < 1 || p->m < 1) return fail(UOT_ERR_ARG, "empty problem");
    if (R < 1) return fail(UOT_ERR_ARG, "R must be >= 1");
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return fail(UOT_ERR_ARG, "eps must be finite and > 0");
    if (!(p->tau > 0.0)) return fail(UOT_ERR_ARG, "tau must be > 0 (or +inf)");
    if (o->max_iter < 1) return fail(UOT_ERR_ARG, "max_iter must be >= 1");
    if (o->tol > 0.0 || o->absorb_log_threshold != 0.0 || records_iterates(o) || o->persistent || o->u0 || o->v0)
        return fail(UOT_ERR_UNSUPPORTED,
                    "the multi-right-hand-side form runs a fixed iteration count with no absorption, "
                    "checkpoints or warm start");
    if (p->k_dtype != UOT_F32 && p->k_dtype != UOT_BF16)
        return fail(UOT_ERR_DTYPE, "the multi-right-hand-side form takes an FP32 or BF16 K");
    if (!p->K) return fail(UOT_ERR_ARG, "K is required");
    M.bf16 = p->k_dtype == UOT_BF16;
    M.es = elem_size(p->k_dtype);
    if (p->ldk < p->m || !aligned(p->K, 16) || p->ldk % (16 / M.es) != 0)
        return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned with ldk >= m a multiple of %d", 16 / M.es);
    if (!(p->k_scale >= 0.0) || !isfinite(p->k_scale)) return fail(UOT_ERR_ARG, "k_scale must be finite and >= 0");
    M.n = p->n;
    M.m = p->m;
    M.R = R;
    M.r_pad = round_up(R, kMTileCols);
    if (M.r_pad > 65535) return fail(UOT_ERR_UNSUPPORTED, "R must be below 65408");
    M.ldn = round_up(p->n, 64);
    M.ldm = round_up(p->m, 64);
    if ((int64_t)M.n * p->ldk * M.es >= ((int64_t)1 << 31) || M.m * M.ldn * M.es >= ((int64_t)1 << 31) ||
        M.r_pad * std::max(M.ldn, M.ldm) * M.es >= ((int64_t)1 << 31))
        return fail(UOT_ERR_UNSUPPORTED, "K and the right-hand sides must each be below 2 GiB");
    // BF16 product kernels (FP32 K always takes the 128 x 128 LDS tiles):
    // tune = 0 (default) or 3: 256 x 256 tiles over a tiled copy of K when R
    // is a multiple of 256 (else as 1; 190 against 208 us per iteration at
    // 8192^2 x 256); 1: 128 x 128 tiles through LDS; 2: per-wave fragment
    // loads; 4: 128 x 128 tiles over the tiled copy
    if (o->tune < 0 || o->tune > 4) return fail(UOT_ERR_ARG, "tune must be 0..4 for the multi-right-hand-side form");
    if (o->tune == 2) M.variant = 0;
    else if (!M.bf16 || o->tune == 1) M.variant = 1;
    else if (o->tune == 0 || o->tune == 3) M.variant = M.r_pad % kMBigCols == 0 ? 3 : 1;
    else M.variant = 4;
    M.row = multi_gemm_shape(M.n, M.ldm, M.r_pad, M.bf16, M.variant);      // S = K V: rows n, reduction over m
    M.col = multi_gemm_shape(M.m, M.ldn, M.r_pad, M.bf16, M.variant);      // W = K^T U: rows m, reduction over n
    // ring variants read K and K^T from tiled copies (launch_mpack)
    M.blocked = M.variant >= 3;
    if (M.blocked && (M.row.rows_pad * M.ldm * 2 >= ((int64_t)1 << 31) || M.col.rows_pad * M.ldn * 2 >= ((int64_t)1 << 31)))
        return fail(UOT_ERR_UNSUPPORTED, "K must be below 2 GiB in the tiled layout");
    size_t off = 0;
    M.off_kt = off;
    off = align_up(off + (M.blocked ? (size_t)M.col.rows_pad * M.ldn * 2 : (size_t)M.m * M.ldn * M.es), kAlign);
    M.off_kb = off;
    if (M.blocked) off = align_up(off + (size_t)M.row.rows_pad * M.ldm * 2, kAlign);
    M.off_part = off;
    const size_t part = std::max((size_t)M.row.splits * M.r_pad * M.row.rows_pad,
                                 (size_t)M.col.splits * M.r_pad * M.col.rows_pad) * sizeof(float);
    off = align_up(off + part, kAlign);
    const int xe = M.bf16 ? 2 : 4;
    M.off_uhi = off;
    off = align_up(off + (size_t)M.r_pad * M.ldn * xe, kAlign);
    M.off_ulo = off;
    if (M.bf16) off = align_up(off + (size_t)M.r_pad * M.ldn * xe, kAlign);
    M.off_vhi = off;
    off = align_up(off + (size_t)M.r_pad * M.ldm * xe, kAlign);
    M.off_vlo = off;
    if (M.bf16) off = align_up(off + (size_t)M.r_pad * M.ldm * xe, kAlign);
    M.off_rm = off;
    off = align_up(off + sizeof(double) * (size_t)R * M.n, kAlign);
    M.off_cm = off;
    off = align_up(off + sizeof(double) * (size_t)R * M.m, kAlign);
    M.off_flags = off;
    off = align_up(off + 64, kAlign);
    M.total = off;
    return UOT_OK;
}

uot_status run_multi(const uot_problem* p, int32_t R, const double* A, const double* B, const uot_options* o,
                     double* U, double* V, double* losses, uot_info* info, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
    MultiPlan M;
    uot_status st = make_multi_plan(p, R, o, M);
    if (st != UOT_OK) return st;
    if (!A || !B || !U || !V || !losses || !info) return fail(UOT_ERR_ARG, "A, B, U, V, losses and info are required");
    if (!aligned(A, 8) || !aligned(B, 8) || !aligned(U, 8) || !aligned(V, 8) || !aligned(losses, 8) || !aligned(info, 8))
        return fail(UOT_ERR_ALIGN, "vectors must be 8-byte aligned");
    if (!ws || ws_bytes < M.total || !aligned(ws, kAlign)) return fail(UOT_ERR_WORKSPACE, "workspace too small or misaligned");
    char* base = (char*)ws;
    void* KT = base + M.off_kt;
    float* part = (float*)(base + M.off_part);
    void* uhi = base + M.off_uhi;
    void* ulo = M.bf16 ? (void*)(base + M.off_ulo) : nullptr;
    void* vhi = base + M.off_vhi;
    void* vlo = M.bf16 ? (void*)(base + M.off_vlo) : nullptr;
    double* Rm = (double*)(base + M.off_rm);
    double* Cm = (double*)(base + M.off_cm);
    uint32_t* flags = (uint32_t*)(base + M.off_flags);
    const double fi = fi_of(p->eps, p->tau);
    const int fi_one = isinf(p->tau) ? 1 : 0;
    const double ks = p->k_scale > 0.0 ? p->k_scale : 1.0;

    UOT_HIP(launch_multi_info(info, 0, flags, 1, stream), "multi reset");
    void* KB = base + M.off_kb;
    if (M.blocked) {
        UOT_HIP(launch_mpack(0, p->K, p->ldk, M.n, M.m, KB, M.row.rows_pad, M.ldm, stream), "tiled K");
        UOT_HIP(launch_mpack(1, p->K, p->ldk, M.n, M.m, KT, M.col.rows_pad, M.ldn, stream), "tiled K^T");
    } else {
        UOT_HIP(launch_transpose(p->k_dtype, p->K, p->ldk, M.n, M.m, KT, M.ldn, stream), "transpose");
    }
    UOT_HIP(launch_ones_rhs(M.bf16, vhi, vlo, R, M.r_pad, M.m, M.ldm, stream), "initial v");

    MGemm rowg;
    memset(&rowg, 0, sizeof(rowg));
    rowg.A = M.blocked ? KB : p->K;
    rowg.blocked = M.blocked;
    rowg.lda = p->ldk;
    rowg.rows = M.n;
    rowg.rows_pad = M.row.rows_pad;
    rowg.kdim_pad = M.row.kdim_pad;
    rowg.x_hi = vhi;
    rowg.x_lo = vlo;
    rowg.ldx = M.ldm;
    rowg.r_pad = M.r_pad;
    rowg.splits = M.row.splits;
    rowg.kchunk = M.row.kchunk;
    rowg.part = part;
    rowg.ld_part = M.row.rows_pad;
    rowg.variant = M.variant;
    MGemm colg = rowg;
    colg.A = KT;
    colg.lda = M.ldn;
    colg.rows = M.m;
    colg.rows_pad = M.col.rows_pad;
    colg.kdim_pad = M.col.kdim_pad;
    colg.x_hi = uhi;
    colg.x_lo = ulo;
    colg.ldx = M.ldn;
    colg.splits = M.col.splits;
    colg.kchunk = M.col.kchunk;
    colg.ld_part = M.col.rows_pad;

    MEpi eu;
    memset(&eu, 0, sizeof(eu));
    eu.part = part;
    eu.ld_part = M.row.rows_pad;
    eu.splits = M.row.splits;
    eu.rows = M.n;
    eu.R = R;
    eu.r_pad = M.r_pad;
    eu.target = A;
    eu.y = U;
    eu.next_hi = uhi;
    eu.next_lo = ulo;
    eu.ld_next = M.ldn;
    eu.bf16 = M.bf16;
    eu.fi = fi;
    eu.fi_is_one = fi_one;
    eu.k_scale = ks;
    eu.mode = 0;
    eu.flags = flags;
    MEpi ev = eu;
    ev.ld_part = M.col.rows_pad;
    ev.splits = M.col.splits;
    ev.rows = M.m;
    ev.target = B;
    ev.y = V;
    ev.next_hi = vhi;
    ev.next_lo = vlo;
    ev.ld_next = M.ldm;

    for (int t = 1; t <= o->max_iter; ++t) {
        eu.store_y = ev.store_y = (t == o->max_iter);      // U and V of the last iteration
        UOT_HIP(launch_mgemm(M.bf16, rowg, stream), "row product");
        UOT_HIP(launch_mepi(eu, stream), "row update");
        UOT_HIP(launch_mgemm(M.bf16, colg, stream), "column product");
        ev.marg = (t == o->max_iter) ? Cm : nullptr;      // c = v (K^T u) of the last iteration
        UOT_HIP(launch_mepi(ev, stream), "column update");
    }
    // r = u (K v) with the final v
    UOT_HIP(launch_mgemm(M.bf16, rowg, stream), "marginal product");
    MEpi er = eu;
    er.mode = 1;
    er.marg = Rm;
    UOT_HIP(launch_mepi(er, stream), "row marginal");
    UOT_HIP(launch_multi_loss(U, V, Rm, Cm, A, B, M.n, M.m, R, p->eps, p->tau, fi_one, losses, flags, stream), "objective");
    UOT_HIP(launch_multi_info(info, o->max_iter, flags, 0, stream), "info");
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
    if (k_dtype != UOT_F64 && k_dtype != UOT_F32 && k_dtype != UOT_BF16 && k_dtype != UOT_FP8_E4M3)
        return fail(UOT_ERR_DTYPE, "K dtype %d not supported", k_dtype);
    int vec = 16 / elem_size(k_dtype);
    if (!aligned(K, 16) || ldk % vec != 0) return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned, ldk a multiple of %d", vec);
    if (!aligned(C, 8)) return fail(UOT_ERR_ALIGN, "C must be 8-byte aligned");
    UOT_HIP(launch_kernel_build(C, ldc, n, m, eps, f, g, k_dtype, K, ldk, k_dtype == UOT_FP8_E4M3 ? 448.0 : 1.0,
                                (hipStream_t)stream),
            "kernel build");
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

uot_status uot_sinkhorn_noalloc(const uot_problem* prob, const uot_options* opt, const uot_outputs* out,
                                void* stream) {
    Plan P;
    uot_status st = make_plan(prob, opt, P);
    if (st != UOT_OK) return st;
    if (P.stab)
        return fail(UOT_ERR_UNSUPPORTED, "the no-allocation entry point runs without absorption (it waits on the host)");
    if (P.total > kScratchBytes)
        return fail(UOT_ERR_WORKSPACE, "problem needs %zu bytes of scratch; the no-allocation entry point holds %zu",
                    P.total, kScratchBytes);
    void* ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != UOT_OK) return st;
    return run_sinkhorn(prob, opt, out, ws, kScratchBytes, (hipStream_t)stream, nullptr, true);
}

uot_status uot_sinkhorn_profiled(const uot_problem* prob, const uot_options* opt, const uot_outputs* out,
                                 void* ws, size_t ws_bytes, void* stream, uot_profile* prof) {
    if (!prof) return fail(UOT_ERR_ARG, "prof must not be NULL");
    return run_sinkhorn(prob, opt, out, ws, ws_bytes, (hipStream_t)stream, prof);
}

uot_status uot_kernel_to_f32(const void* K, int32_t k_dtype, int64_t count, double k_scale, float* out,
                             void* stream) {
    if (!K || !out || count < 0) return fail(UOT_ERR_ARG, "K and out must not be NULL, count >= 0");
    const int es = elem_size(k_dtype);
    if (es == 0) return fail(UOT_ERR_DTYPE, "unknown dtype %d", k_dtype);
    if (count % (16 / es) != 0) return fail(UOT_ERR_ALIGN, "count must be a multiple of %d", 16 / es);
    if (!aligned(K, 16)) return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned");
    UOT_HIP(launch_decode(K, k_dtype, count, k_scale, out, (hipStream_t)stream), "decode");
    return UOT_OK;
}

size_t uot_sinkhorn_backward_workspace_size(const uot_problem* prob, const uot_options* opt, int64_t dim,
                                            int32_t cost_grad) {
    BwdPlan B;
    if (make_bwd_plan(prob, opt, dim, cost_grad != 0, B) != UOT_OK) return 0;
    return B.total;
}

uot_status uot_sinkhorn_backward(const uot_problem* prob, const uot_options* opt, const double* u, const double* v,
                                 const double* ckpt, const double* grad_loss, double* grad_a, double* grad_b,
                                 double* grad_C, int64_t ldgc, const double* x, const double* y, int64_t dim,
                                 double* grad_x, double* grad_y, void* ws, size_t ws_bytes, void* stream) {
    return run_backward(prob, opt, u, v, ckpt, grad_loss, grad_a, grad_b, grad_C, ldgc, x, y, dim, grad_x, grad_y,
                        ws, ws_bytes, (hipStream_t)stream);
}

size_t uot_sinkhorn_points_workspace_size(const uot_problem* prob, int64_t dim, double cost_scale,
                                          const uot_options* opt) {
    PtsPlan P;
    if (make_points_plan(prob, dim, cost_scale, opt, P) != UOT_OK) return 0;
    return P.total;
}

uot_status uot_sinkhorn_points(const uot_problem* prob, const double* x, const double* y, int64_t dim,
                               double cost_scale, const uot_options* opt, const uot_outputs* out, void* ws,
                               size_t ws_bytes, void* stream) {
    return run_points(prob, x, y, dim, cost_scale, opt, out, ws, ws_bytes, (hipStream_t)stream);
}

size_t uot_sinkhorn_lse_workspace_size(const uot_problem* prob, const uot_options* opt, const uot_eps_schedule* sched) {
    LsePlan P;
    if (make_lse_plan(prob, opt, sched, P) != UOT_OK) return 0;
    return P.total;
}

uot_status uot_sinkhorn_lse(const uot_problem* prob, const uot_options* opt, const uot_eps_schedule* sched,
                            const uot_outputs* out, void* ws, size_t ws_bytes, void* stream) {
    return run_lse(prob, opt, sched, out, ws, ws_bytes, (hipStream_t)stream);
}

size_t uot_matrix_rescale_workspace_size(const uot_problem* prob, const uot_options* opt) {
    Plan P;
    if (make_matrix_plan(prob, opt, P) != UOT_OK) return 0;
    return P.total;
}

uot_status uot_matrix_rescale(const uot_problem* prob, const uot_options* opt, const uot_outputs* out, void* ws,
                              size_t ws_bytes, void* stream) {
    return run_matrix(prob, opt, out, ws, ws_bytes, (hipStream_t)stream);
}

size_t uot_sinkhorn_implicit_backward_workspace_size(const uot_problem* prob, const uot_options* opt, int64_t dim) {
    ImpPlan B;
    if (make_imp_plan(prob, opt, dim, B) != UOT_OK) return 0;
    return B.total;
}

uot_status uot_sinkhorn_implicit_backward(const uot_problem* prob, const uot_options* opt, const double* u,
                                          const double* v, const double* grad_loss, double* grad_a, double* grad_b,
                                          double* grad_C, int64_t ldgc, const double* x, const double* y, int64_t dim,
                                          double* grad_x, double* grad_y, void* ws, size_t ws_bytes, void* stream) {
    return run_implicit_backward(prob, opt, u, v, grad_loss, grad_a, grad_b, grad_C, ldgc, x, y, dim, grad_x, grad_y,
                                 ws, ws_bytes, (hipStream_t)stream);
}

size_t uot_batched_desc_bytes(int32_t count) { return count < 0 ? 0 : batch_desc_bytes(count) + sizeof(uot_batched_meta); }

uot_status uot_batched_pack(const uot_problem* probs, int32_t count, const uot_options* opt,
                            const uot_outputs* outs, void* desc_host, size_t desc_bytes) {
    if (!desc_host) return fail(UOT_ERR_ARG, "desc_host must not be NULL");
    if (count < 0 || desc_bytes < uot_batched_desc_bytes(count)) return fail(UOT_ERR_ARG, "desc_bytes too small");
    BatchPack pk;
    uot_status st = pack_batch(probs, count, opt, outs, true, pk);
    if (st != UOT_OK) return st;
    memset(desc_host, 0, desc_bytes);
    if (!pk.d.empty()) memcpy(desc_host, pk.d.data(), sizeof(BatchDesc) * pk.d.size());
    uot_batched_meta meta;
    memset(&meta, 0, sizeof(meta));
    meta.count = count;
    meta.k_dtype = count > 0 ? probs[0].k_dtype : UOT_F32;
    meta.m_lds = pk.m_lds;
    meta.items = (int32_t)pk.d.size();
    meta.nsplit = pk.nsplit;
    meta.pool_bytes = (int64_t)pk.pool_used;
    memcpy((char*)desc_host + batch_desc_bytes(count), &meta, sizeof(meta));
    return UOT_OK;
}

size_t uot_sinkhorn_batched_workspace_size(int32_t count) {
    if (count < 0) return 0;
    return kAlign + batch_desc_bytes(count) + batch_pool_bytes(count);
}

uot_status uot_sinkhorn_batched_packed(const void* desc_dev, const uot_batched_meta* meta, const uot_options* opt,
                                       void* ws, size_t ws_bytes, uint64_t* trace, void* stream) {
    if (!meta) return fail(UOT_ERR_ARG, "meta must not be NULL");
    uot_status st = check_batch_options(opt);
    if (st != UOT_OK) return st;
    if (meta->count < 0 || (meta->count > 0 && !desc_dev)) return fail(UOT_ERR_ARG, "bad descriptor block");
    if (meta->items < meta->count || meta->items > batch_max_items(meta->count) || meta->nsplit < 0 ||
        meta->nsplit > batch_max_splits(meta->count) || meta->pool_bytes < 0 ||
        (size_t)meta->pool_bytes > batch_pool_bytes(meta->count))
        return fail(UOT_ERR_ARG, "bad descriptor block meta (items, splits or pool size)");
    if (!aligned(desc_dev, 16)) return fail(UOT_ERR_ALIGN, "descriptors must be 16-byte aligned");
    if (elem_size(meta->k_dtype) == 0) return fail(UOT_ERR_DTYPE, "bad K dtype in meta");
    if (trace && !aligned(trace, 8)) return fail(UOT_ERR_ALIGN, "trace must be 8-byte aligned");
    return run_batch_packed((const BatchDesc*)desc_dev, meta->items, meta->nsplit, batch_desc_bytes(meta->count),
                            (size_t)meta->pool_bytes, meta->k_dtype, meta->m_lds, opt, ws, ws_bytes, trace,
                            (hipStream_t)stream);
}

uot_status uot_sinkhorn_batched(const uot_problem* probs, int32_t count, const uot_options* opt,
                                const uot_outputs* outs, void* ws, size_t ws_bytes, void* stream) {
    if (count < 0) return fail(UOT_ERR_ARG, "count must be >= 0");
    if (count == 0) return check_batch_options(opt);
    if (!ws || ws_bytes < uot_sinkhorn_batched_workspace_size(count) || !aligned(ws, kAlign))
        return fail(UOT_ERR_WORKSPACE, "workspace too small or misaligned");
    hipStream_t s = (hipStream_t)stream;
    if (opt && opt->tune > 0 && probs) {
        uot_status st = autotune_batch(probs, count, opt, outs, ws, ws_bytes, s);
        if (st != UOT_OK) return st;
    }
    BatchPack pk;
    uot_status st = pack_batch(probs, count, opt, outs, true, pk);
    if (st != UOT_OK) return st;
    BatchDesc* ddev = (BatchDesc*)((char*)ws + kAlign);
    // pageable source: the copy has consumed it when the call returns
    UOT_HIP(hipMemcpyAsync(ddev, pk.d.data(), sizeof(BatchDesc) * pk.d.size(), hipMemcpyHostToDevice, s),
            "descriptor copy");
    UOT_HIP(hipStreamSynchronize(s), "descriptor copy");
    return run_batch_packed(ddev, (int32_t)pk.d.size(), pk.nsplit, batch_desc_bytes(count), pk.pool_used,
                            probs[0].k_dtype, pk.m_lds, opt, ws, ws_bytes, nullptr, s);
}

uot_status uot_batched_tune(const uot_problem* probs, int32_t count, const uot_options* opt, const uot_outputs* outs,
                            void* ws, size_t ws_bytes, void* stream) {
    if (count <= 0) return UOT_OK;
    if (!probs || !outs) return fail(UOT_ERR_ARG, "probs and outs must not be NULL");
    uot_status st = check_batch_options(opt);
    if (st != UOT_OK) return st;
    if (!ws || ws_bytes < uot_sinkhorn_batched_workspace_size(std::min(count, 8)) || !aligned(ws, kAlign))
        return fail(UOT_ERR_WORKSPACE, "workspace too small or misaligned");
    return autotune_batch(probs, count, opt, outs, ws, ws_bytes, (hipStream_t)stream);
}

int64_t uot_device_wall_clock_khz(void) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return v;
}

uot_status uot_plan(const uot_problem* prob, const double* u, const double* v, const double* f, const double* g,
                    void* plan, int64_t ldp, int32_t plan_dtype, void* stream) {
    if (!prob || !plan) return fail(UOT_ERR_ARG, "problem and plan must not be NULL");
    if (prob->n < 1 || prob->m < 1) return fail(UOT_ERR_ARG, "empty problem");
    if (plan_dtype != UOT_F64 && plan_dtype != UOT_F32) return fail(UOT_ERR_DTYPE, "plan dtype must be F64 or F32");
    if (ldp < prob->m) return fail(UOT_ERR_ARG, "ldp (%lld) < m (%lld)", (long long)ldp, (long long)prob->m);
    if (!aligned(plan, elem_size(plan_dtype))) return fail(UOT_ERR_ALIGN, "plan misaligned");
    hipStream_t s = (hipStream_t)stream;
    if (prob->K && u && v) {
        const int es = elem_size(prob->k_dtype);
        if (es == 0) return fail(UOT_ERR_DTYPE, "K dtype %d not supported", (int)prob->k_dtype);
        if (prob->ldk < prob->m) return fail(UOT_ERR_ARG, "ldk < m");
        if (!aligned(prob->K, 16) || prob->ldk % (16 / es) != 0)
            return fail(UOT_ERR_ALIGN, "K must be 16-byte aligned with ldk a multiple of %d", 16 / es);
        if (!aligned(u, 8) || !aligned(v, 8)) return fail(UOT_ERR_ALIGN, "u and v must be 8-byte aligned");
        const double ks = prob->k_scale > 0.0 ? prob->k_scale : 1.0;
        UOT_HIP(launch_plan_from_k(prob->K, prob->k_dtype, prob->ldk, prob->n, prob->m, ks, u, v, plan, plan_dtype,
                                   ldp, s), "plan");
        return UOT_OK;
    }
    if (prob->C && f && g) {
        if (prob->ldc < prob->m) return fail(UOT_ERR_ARG, "ldc < m");
        if (!(prob->eps > 0.0)) return fail(UOT_ERR_ARG, "eps must be > 0");
        if (!aligned(prob->C, 8) || !aligned(f, 8) || !aligned(g, 8)) return fail(UOT_ERR_ALIGN, "C, f, g must be 8-byte aligned");
        UOT_HIP(launch_plan_from_cost(prob->C, prob->ldc, prob->n, prob->m, prob->eps, f, g, plan, plan_dtype, ldp, s),
                "plan");
        return UOT_OK;
    }
    return fail(UOT_ERR_ARG, "the plan needs K with u and v, or C with f and g");
}

size_t uot_sinkhorn_multi_workspace_size(const uot_problem* shared, int32_t R, const uot_options* opt) {
    MultiPlan M;
    if (make_multi_plan(shared, R, opt, M) != UOT_OK) return 0;
    return M.total;
}

uot_status uot_sinkhorn_multi(const uot_problem* shared, int32_t R, const double* A, const double* B,
                              const uot_options* opt, double* U, double* V, double* losses, uot_info* info, void* ws,
                              size_t ws_bytes, void* stream) {
    return run_multi(shared, R, A, B, opt, U, V, losses, info, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
