/*
 * FP64 CPU oracle for the entropic unbalanced optimal-transport (UOT)
 * Sinkhorn scaling loop -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct definition that the HIP
 * library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it; the product path never does.  It
 * shares no source, header, table or helper with the HIP library.
 *
 * Problem (paper Section 2.1): a non-negative matrix is rescaled
 * alternately by rows and by columns; the row factor of row i is
 * (row target_i / row sum_i)^fi with fi = tau/(tau+eps) (the paper's
 * fi = er/(er+ep)), and likewise for columns, until an error limit.  Written
 * on scaling vectors (the form used here), the kernel is K = exp(-C/eps),
 * the plan is P = diag(u) K diag(v), and one iteration is
 *
 *     s = K v,      u = (a / s)^fi          (row half-step: parts 4 and 1
 *     w = K^T u,    v = (b / w)^fi           and column half-step: parts 2, 3
 *                                            of the four-part split, Sec. 4)
 *
 * rows first, starting from v = 1.  Every routine below is FP64, uses no
 * blocking or reordering beyond what that definition states, and is
 * parallelised only across independent rows or independent column blocks
 * (each output element is summed in ascending index order, so results do
 * not depend on the thread count).
 *
 * Readings where the paper is silent (each is listed with its reason in
 * the design notes):
 *   - zero mass: a_i = 0 gives u_i = 0 (and b_j = 0 gives v_j = 0), even
 *     when the sum is 0; a zero sum with positive mass yields +inf (the
 *     caller sees it as non-finite);
 *   - stopping: the error after iteration t is the relative L1 change of
 *     the column marginal c_t = v_t * (K^T u_t), with c_0 = 0; stop when
 *     tol > 0 and the error is <= tol, otherwise run exactly max_iter;
 *   - objective: the primal UOT objective
 *        <C,P> + eps sum P (log P - 1) + tau KL~(P1|a) + tau KL~(P^T1|b),
 *     KL~(x|y) = sum x log(x/y) - x + y, 0 log 0 = 0; for tau = inf the two
 *     KL terms are dropped.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* Exponent of the row/column factors (Section 2.1): tau/(tau+eps), or 1 for
 * the balanced limit tau = inf. */
static double orc_fi(double eps, double tau) {
    if (isinf(tau)) return 1.0;
    return tau / (tau + eps);
}

/* One scaling factor (target / sum)^fi with the zero-mass rule. */
static double orc_factor(double target, double sum, double fi) {
    if (target == 0.0) return 0.0;
    return pow(target / sum, fi);
}

/* ------------------------------------------------------------------ */
/* Costs and kernel                                                     */
/* ------------------------------------------------------------------ */

/* C_ij = ||x_i - y_j||^2 (kind 0) or 1 - x_i . y_j (kind 1); x is n x d,
 * y is m x d, both row-major; C is n x m row-major.  With normalize != 0
 * the whole matrix is divided by its maximum (if that maximum is > 0). */
ORC_EXPORT void orc_cost_points(const double* x, const double* y, int64_t n, int64_t m,
                                int64_t d, int kind, int normalize, double* C) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double acc = 0.0;
            if (kind == 0) {
                for (int64_t k = 0; k < d; ++k) {
                    double diff = x[i * d + k] - y[j * d + k];
                    acc += diff * diff;
                }
                C[i * m + j] = acc;
            } else {
                for (int64_t k = 0; k < d; ++k) acc += x[i * d + k] * y[j * d + k];
                C[i * m + j] = 1.0 - acc;
            }
        }
    }
    if (normalize) {
        double mx = 0.0;
        for (int64_t t = 0; t < n * m; ++t) if (C[t] > mx) mx = C[t];
        if (mx > 0.0) {
            #pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < n * m; ++t) C[t] = C[t] / mx;
        }
    }
}

/* K_ij = exp((f_i + g_j - C_ij) / eps); f or g may be NULL (taken as 0).
 * With f = g = 0 this is the Gibbs kernel exp(-C/eps). */
ORC_EXPORT void orc_kernel(const double* C, int64_t n, int64_t m, double eps,
                           const double* f, const double* g, double* K) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fi_ = f ? f[i] : 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double gj = g ? g[j] : 0.0;
            K[i * m + j] = exp((fi_ + gj - C[i * m + j]) / eps);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Mat-vec products                                                     */
/* ------------------------------------------------------------------ */

/* s = K v (row sums of diag(.) K diag(v)). */
static void orc_Kv(const double* K, const double* v, int64_t n, int64_t m, double* s) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) acc += K[i * m + j] * v[j];
        s[i] = acc;
    }
}

/* w = K^T u, each w_j summed over i in ascending order; threads own blocks
 * of 64 columns so that rows are still read in contiguous pieces. */
static void orc_KTu(const double* K, const double* u, int64_t n, int64_t m, double* w) {
    const int64_t BLK = 64;
    int64_t nblk = (m + BLK - 1) / BLK;
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t j0 = blk * BLK, j1 = j0 + BLK < m ? j0 + BLK : m;
        double acc[64];
        for (int64_t j = j0; j < j1; ++j) acc[j - j0] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double ui = u[i];
            const double* row = K + i * m;
            for (int64_t j = j0; j < j1; ++j) acc[j - j0] += row[j] * ui;
        }
        for (int64_t j = j0; j < j1; ++j) w[j] = acc[j - j0];
    }
}

/* ------------------------------------------------------------------ */
/* Plain Sinkhorn (vector form, rows first)                             */
/* ------------------------------------------------------------------ */

/*
 * Runs the iteration from v = v0 (or 1) for at most max_iter iterations.
 * Outputs (all caller-allocated, length n or m):
 *   u, v          final scalings u_T, v_T (u = 1 when max_iter = 0 and no u0)
 *   s_fin         K v_T            (so the row marginal is r = u * s_fin)
 *   w_fin         K^T u_T          (so the column marginal is c = v * w_fin)
 *   err_out       error of the last iteration run (0 when none was run)
 * Optional trace (NULL to skip), for the reverse pass:
 *   tr_v  (max_iter+1) x m : v_0 .. v_T
 *   tr_s  max_iter x n      : s_1 .. s_T     (s_t = K v_{t-1})
 *   tr_u  max_iter x n      : u_1 .. u_T
 *   tr_w  max_iter x m      : w_1 .. w_T     (w_t = K^T u_t)
 * Returns the number of iterations run.
 */
ORC_EXPORT int64_t orc_sinkhorn(const double* K, const double* a, const double* b,
                                int64_t n, int64_t m, double eps, double tau,
                                int64_t max_iter, double tol,
                                const double* u0, const double* v0,
                                double* u, double* v, double* s_fin, double* w_fin,
                                double* err_out,
                                double* tr_v, double* tr_s, double* tr_u, double* tr_w) {
    double fi = orc_fi(eps, tau);
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    double* c_prev = (double*)calloc((size_t)m, sizeof(double));
    for (int64_t i = 0; i < n; ++i) u[i] = u0 ? u0[i] : 1.0;
    for (int64_t j = 0; j < m; ++j) v[j] = v0 ? v0[j] : 1.0;
    if (tr_v) memcpy(tr_v, v, sizeof(double) * (size_t)m);
    double err = 0.0;
    int64_t t = 0;
    while (t < max_iter) {
        /* row half-step */
        orc_Kv(K, v, n, m, s);
        for (int64_t i = 0; i < n; ++i) u[i] = orc_factor(a[i], s[i], fi);
        /* column half-step */
        orc_KTu(K, u, n, m, w);
        for (int64_t j = 0; j < m; ++j) v[j] = orc_factor(b[j], w[j], fi);
        ++t;
        if (tr_s) memcpy(tr_s + (t - 1) * n, s, sizeof(double) * (size_t)n);
        if (tr_u) memcpy(tr_u + (t - 1) * n, u, sizeof(double) * (size_t)n);
        if (tr_w) memcpy(tr_w + (t - 1) * m, w, sizeof(double) * (size_t)m);
        if (tr_v) memcpy(tr_v + t * m, v, sizeof(double) * (size_t)m);
        /* relative L1 change of the column marginal c = v * w */
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double cj = v[j] * w[j];
            num += fabs(cj - c_prev[j]);
            den += fabs(cj);
            c_prev[j] = cj;
        }
        err = num / den;
        if (tol > 0.0 && err <= tol) break;
    }
    orc_Kv(K, v, n, m, s_fin);
    orc_KTu(K, u, n, m, w_fin);
    if (err_out) *err_out = err;
    free(s);
    free(w);
    free(c_prev);
    return t;
}

/* ------------------------------------------------------------------ */
/* Objective                                                            */
/* ------------------------------------------------------------------ */

/* KL~(x|y) = x log(x/y) - x + y with 0 log 0 = 0. */
static double orc_kl_term(double x, double y) {
    double t = -x + y;
    if (x > 0.0) t += x * log(x / y);
    return t;
}

/*
 * Primal objective by its definition, summing over all n x m entries of
 * P = diag(u) K diag(v):  <C,P> + eps sum P(log P - 1) + tau KL~(r|a)
 * + tau KL~(c|b), with r = P 1 and c = P^T 1 formed here from P.
 * transport_cost (optional) receives <C,P>.
 */
ORC_EXPORT double orc_loss_direct(const double* C, const double* K, const double* u,
                                  const double* v, const double* a, const double* b,
                                  int64_t n, int64_t m, double eps, double tau,
                                  double* transport_cost) {
    double* r = (double*)calloc((size_t)n, sizeof(double));
    double* c = (double*)calloc((size_t)m, sizeof(double));
    double cp = 0.0, ent = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double p = u[i] * K[i * m + j] * v[j];
            r[i] += p;
            c[j] += p;
            cp += C[i * m + j] * p;
            if (p > 0.0) ent += p * (log(p) - 1.0);
        }
    }
    double L = cp + eps * ent;
    if (!isinf(tau)) {
        double kr = 0.0, kc = 0.0;
        for (int64_t i = 0; i < n; ++i) kr += orc_kl_term(r[i], a[i]);
        for (int64_t j = 0; j < m; ++j) kc += orc_kl_term(c[j], b[j]);
        L += tau * (kr + kc);
    }
    if (transport_cost) *transport_cost = cp;
    free(r);
    free(c);
    return L;
}

/*
 * The same objective from O(n + m) quantities.  Because
 * eps log P_ij = eps log u_i + eps log v_j - C_ij, the cost and entropy
 * terms collapse to eps (sum r log u + sum c log v - sum r); r = u * (K v)
 * and c = v * (K^T u) are passed in.
 */
ORC_EXPORT double orc_loss_identity(const double* u, const double* v, const double* r,
                                    const double* c, const double* a, const double* b,
                                    int64_t n, int64_t m, double eps, double tau) {
    double sr = 0.0, sc = 0.0, mass = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (r[i] > 0.0) sr += r[i] * log(u[i]);
        mass += r[i];
    }
    for (int64_t j = 0; j < m; ++j)
        if (c[j] > 0.0) sc += c[j] * log(v[j]);
    double L = eps * (sr + sc - mass);
    if (!isinf(tau)) {
        double kr = 0.0, kc = 0.0;
        for (int64_t i = 0; i < n; ++i) kr += orc_kl_term(r[i], a[i]);
        for (int64_t j = 0; j < m; ++j) kc += orc_kl_term(c[j], b[j]);
        L += tau * (kr + kc);
    }
    return L;
}

/* ------------------------------------------------------------------ */
/* Stabilised (absorbed) iteration                                      */
/* ------------------------------------------------------------------ */

/*
 * The same iterates written on (f, g, u, v) with total scalings
 * U = u e^{f/eps}, V = v e^{g/eps} and the rescaled kernel
 * Kt_ij = exp((f_i + g_j - C_ij)/eps):
 *     u = (a / (Kt v))^fi * exp(-(1-fi) f / eps)
 *     v = (b / (Kt^T u))^fi * exp(-(1-fi) g / eps)
 * After each half-step, if max|log u| or max|log v| exceeds threshold
 * (> 0), both are absorbed (f += eps log u, g += eps log v, u = v = 1) and
 * Kt is rebuilt.  Initial f_i = min_j C_ij, g = 0 (an exact
 * reparameterisation: it only moves scale between u and Kt).
 * Outputs f, g (final potentials of the total scalings, i.e. including the
 * residual u, v), the residual u, v are folded in.  Returns iterations;
 * *absorptions receives the number of absorptions.
 */
ORC_EXPORT int64_t orc_sinkhorn_stabilized(const double* C, const double* a, const double* b,
                                           int64_t n, int64_t m, double eps, double tau,
                                           int64_t max_iter, double threshold,
                                           double* f, double* g, int64_t* absorptions) {
    double fi = orc_fi(eps, tau);
    double* Kt = (double*)malloc(sizeof(double) * (size_t)(n * m));
    double* u = (double*)malloc(sizeof(double) * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * (size_t)m);
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t i = 0; i < n; ++i) {
        double mn = INFINITY;
        for (int64_t j = 0; j < m; ++j) if (C[i * m + j] < mn) mn = C[i * m + j];
        f[i] = mn;
        u[i] = 1.0;
    }
    for (int64_t j = 0; j < m; ++j) { g[j] = 0.0; v[j] = 1.0; }
    orc_kernel(C, n, m, eps, f, g, Kt);
    int64_t nabs = 0;
    for (int64_t t = 0; t < max_iter; ++t) {
        orc_Kv(Kt, v, n, m, s);
        for (int64_t i = 0; i < n; ++i)
            u[i] = (a[i] == 0.0) ? 0.0
                 : pow(a[i] / s[i], fi) * exp(-(1.0 - fi) * f[i] / eps);
        orc_KTu(Kt, u, n, m, w);
        for (int64_t j = 0; j < m; ++j)
            v[j] = (b[j] == 0.0) ? 0.0
                 : pow(b[j] / w[j], fi) * exp(-(1.0 - fi) * g[j] / eps);
        if (threshold > 0.0) {
            double mx = 0.0;
            for (int64_t i = 0; i < n; ++i) if (u[i] > 0.0 && fabs(log(u[i])) > mx) mx = fabs(log(u[i]));
            for (int64_t j = 0; j < m; ++j) if (v[j] > 0.0 && fabs(log(v[j])) > mx) mx = fabs(log(v[j]));
            if (mx > threshold) {
                for (int64_t i = 0; i < n; ++i) { if (u[i] > 0.0) f[i] += eps * log(u[i]); u[i] = 1.0; }
                for (int64_t j = 0; j < m; ++j) { if (v[j] > 0.0) g[j] += eps * log(v[j]); v[j] = 1.0; }
                orc_kernel(C, n, m, eps, f, g, Kt);
                ++nabs;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) f[i] = (u[i] > 0.0) ? f[i] + eps * log(u[i]) : -INFINITY;
    for (int64_t j = 0; j < m; ++j) g[j] = (v[j] > 0.0) ? g[j] + eps * log(v[j]) : -INFINITY;
    if (absorptions) *absorptions = nabs;
    free(Kt); free(u); free(v); free(s); free(w);
    return max_iter;
}

/* ------------------------------------------------------------------ */
/* Reverse mode through the unrolled iteration                          */
/* ------------------------------------------------------------------ */

/*
 * Exact gradient of the objective (identity form, as a function of K, a, b
 * through the T unrolled iterations from v_0 = 1) by reverse-mode
 * differentiation.  Uses the forward trace written by orc_sinkhorn.
 *
 * Seeds, with r = u_T * (K v_T), c = v_T * (K^T u_T):
 *   rbar = eps log u + tau log(r/a) - eps,   cbar = eps log v + tau log(c/b)
 *   ubar = eps r/u + rbar * (K v) + K (cbar * v)
 *   vbar = eps c/v + K^T (rbar * u) + cbar * (K^T u)
 *   Kbar = (rbar * u) v^T + u (cbar * v)^T
 *   abar = tau (1 - r/a),  bbar = tau (1 - c/b)          (tau = inf: 0, and
 *                                                         the log(r/a) terms drop)
 * Then for t = T..1:
 *   wbar = -fi vbar * v_t / w_t;  bbar += fi vbar * v_t / b
 *   ubar += K wbar;               Kbar += u_t wbar^T
 *   sbar = -fi ubar * u_t / s_t;  abar += fi ubar * u_t / a
 *   vbar  = K^T sbar;             Kbar += sbar v_{t-1}^T;   ubar = 0
 * Outputs: grad_a (n), grad_b (m), and G = dL/dC = -Kbar * K / eps (n x m,
 * optional, NULL to skip).  Zero-mass entries are not supported here.
 */
ORC_EXPORT void orc_adjoint(const double* K, const double* a, const double* b,
                            int64_t n, int64_t m, double eps, double tau, int64_t T,
                            const double* tr_v, const double* tr_s, const double* tr_u,
                            const double* tr_w, double* grad_a, double* grad_b, double* G) {
    double fi = orc_fi(eps, tau);
    int bal = isinf(tau);
    const double* uT = tr_u + (T - 1) * n;
    const double* vT = tr_v + T * m;
    double* Kbar = (double*)calloc((size_t)(n * m), sizeof(double));
    double* sv = (double*)malloc(sizeof(double) * (size_t)n);   /* K v_T */
    double* wu = (double*)malloc(sizeof(double) * (size_t)m);   /* K^T u_T */
    double* rbar = (double*)malloc(sizeof(double) * (size_t)n);
    double* cbar = (double*)malloc(sizeof(double) * (size_t)m);
    double* ubar = (double*)malloc(sizeof(double) * (size_t)n);
    double* vbar = (double*)malloc(sizeof(double) * (size_t)m);
    double* tmpn = (double*)malloc(sizeof(double) * (size_t)n);
    double* tmpm = (double*)malloc(sizeof(double) * (size_t)m);
    double* wbar = (double*)malloc(sizeof(double) * (size_t)m);
    double* sbar = (double*)malloc(sizeof(double) * (size_t)n);

    orc_Kv(K, vT, n, m, sv);
    orc_KTu(K, uT, n, m, wu);
    for (int64_t i = 0; i < n; ++i) {
        double r = uT[i] * sv[i];
        rbar[i] = eps * log(uT[i]) - eps + (bal ? 0.0 : tau * log(r / a[i]));
        grad_a[i] = bal ? 0.0 : tau * (1.0 - r / a[i]);
    }
    for (int64_t j = 0; j < m; ++j) {
        double c = vT[j] * wu[j];
        cbar[j] = eps * log(vT[j]) + (bal ? 0.0 : tau * log(c / b[j]));
        grad_b[j] = bal ? 0.0 : tau * (1.0 - c / b[j]);
    }
    /* ubar = eps r/u + rbar*(K v) + K (cbar*v) ; note eps r/u = eps (K v) */
    for (int64_t j = 0; j < m; ++j) tmpm[j] = cbar[j] * vT[j];
    orc_Kv(K, tmpm, n, m, tmpn);
    for (int64_t i = 0; i < n; ++i) ubar[i] = eps * sv[i] + rbar[i] * sv[i] + tmpn[i];
    /* vbar = eps c/v + K^T(rbar*u) + cbar*(K^T u) ; eps c/v = eps (K^T u) */
    for (int64_t i = 0; i < n; ++i) tmpn[i] = rbar[i] * uT[i];
    orc_KTu(K, tmpn, n, m, tmpm);
    for (int64_t j = 0; j < m; ++j) vbar[j] = eps * wu[j] + tmpm[j] + cbar[j] * wu[j];
    /* Kbar = (rbar*u) v^T + u (cbar*v)^T */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j)
            Kbar[i * m + j] = rbar[i] * uT[i] * vT[j] + uT[i] * cbar[j] * vT[j];

    for (int64_t t = T; t >= 1; --t) {
        const double* vt = tr_v + t * m;
        const double* vprev = tr_v + (t - 1) * m;
        const double* st = tr_s + (t - 1) * n;
        const double* ut = tr_u + (t - 1) * n;
        const double* wt = tr_w + (t - 1) * m;
        for (int64_t j = 0; j < m; ++j) {
            wbar[j] = (vt[j] == 0.0) ? 0.0 : -fi * vbar[j] * vt[j] / wt[j];
            if (b[j] != 0.0) grad_b[j] += fi * vbar[j] * vt[j] / b[j];
        }
        orc_Kv(K, wbar, n, m, tmpn);
        for (int64_t i = 0; i < n; ++i) ubar[i] += tmpn[i];
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) Kbar[i * m + j] += ut[i] * wbar[j];
        for (int64_t i = 0; i < n; ++i) {
            sbar[i] = (ut[i] == 0.0) ? 0.0 : -fi * ubar[i] * ut[i] / st[i];
            if (a[i] != 0.0) grad_a[i] += fi * ubar[i] * ut[i] / a[i];
        }
        orc_KTu(K, sbar, n, m, vbar);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) Kbar[i * m + j] += sbar[i] * vprev[j];
        for (int64_t i = 0; i < n; ++i) ubar[i] = 0.0;
    }
    if (G) {
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n * m; ++t) G[t] = -Kbar[t] * K[t] / eps;
    }
    free(Kbar); free(sv); free(wu); free(rbar); free(cbar); free(ubar); free(vbar);
    free(tmpn); free(tmpm); free(wbar); free(sbar);
}

/* Gradient with respect to the source points of a squared-Euclidean cost
 * (not max-normalised): dL/dx_i = 2 sum_j G_ij (x_i - y_j). */
ORC_EXPORT void orc_grad_points_sqeuclid(const double* G, const double* x, const double* y,
                                         int64_t n, int64_t m, int64_t d, double* grad_x) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = 0; k < d; ++k) {
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j) acc += G[i * m + j] * (x[i * d + k] - y[j * d + k]);
            grad_x[i * d + k] = 2.0 * acc;
        }
    }
}

/* Gradient with respect to the target points of the same cost:
 * dL/dy_j = 2 sum_i G_ij (y_j - x_i) (C_ij depends on y_j through
 * ||x_i - y_j||^2, whose derivative in y_j is 2 (y_j - x_i)). */
ORC_EXPORT void orc_grad_target_sqeuclid(const double* G, const double* x, const double* y,
                                         int64_t n, int64_t m, int64_t d, double* grad_y) {
    const int64_t BLK = 64;
    int64_t nblk = (m + BLK - 1) / BLK;
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t j0 = blk * BLK, j1 = j0 + BLK < m ? j0 + BLK : m;
        for (int64_t j = j0; j < j1; ++j)
            for (int64_t k = 0; k < d; ++k) grad_y[j * d + k] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j)
                for (int64_t k = 0; k < d; ++k)
                    grad_y[j * d + k] += G[i * m + j] * (y[j * d + k] - x[i * d + k]);
        for (int64_t j = j0; j < j1; ++j)
            for (int64_t k = 0; k < d; ++k) grad_y[j * d + k] *= 2.0;
    }
}

/* ------------------------------------------------------------------ */
/* The paper's literal in-place matrix rescaling                        */
/* ------------------------------------------------------------------ */
/* Section 2.1's rescaling applied to the matrix itself, in the order of the
 * interleaved single-pass algorithm of Section 4.1 (Algorithm 1: column
 * factors first, then each row).  Before the first iteration the column
 * factors are computed from A's column sums; each iteration then, for every
 * row i: multiplies the row by the column factors, sums it, forms the row
 * factor (RPD_i / sum)^fi, multiplies the row by it and adds the row into
 * the next column sums; at its end the column factors become
 * (CPD_j / column sum_j)^fi.  A (n x m, row-major) is rescaled in place for
 * T iterations; r and c (optional) receive its row and column sums after
 * the last one.  RPD = a, CPD = b; a zero target gives a zero factor.
 * Plain loops, every sum in ascending index order. */
ORC_EXPORT void orc_matrix_rescale(double* A, const double* a, const double* b, int64_t n, int64_t m,
                                   double eps, double tau, int64_t T, double* r, double* c) {
    const double fi = orc_fi(eps, tau);
    double* fcol = (double*)malloc(sizeof(double) * (size_t)m);
    double* next = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t j = 0; j < m; ++j) fcol[j] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) fcol[j] += A[i * m + j];
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t j = 0; j < m; ++j) {
            fcol[j] = orc_factor(b[j], fcol[j], fi);
            next[j] = 0.0;
        }
        for (int64_t i = 0; i < n; ++i) {
            double* row = A + i * m;
            double sum = 0.0;
            for (int64_t j = 0; j < m; ++j) {
                row[j] *= fcol[j];
                sum += row[j];
            }
            const double frow = orc_factor(a[i], sum, fi);
            for (int64_t j = 0; j < m; ++j) {
                row[j] *= frow;
                next[j] += row[j];
            }
        }
        for (int64_t j = 0; j < m; ++j) fcol[j] = next[j];
    }
    if (r)
        for (int64_t i = 0; i < n; ++i) {
            double sum = 0.0;
            for (int64_t j = 0; j < m; ++j) sum += A[i * m + j];
            r[i] = sum;
        }
    if (c) {
        for (int64_t j = 0; j < m; ++j) c[j] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) c[j] += A[i * m + j];
    }
    free(fcol);
    free(next);
}

/* ------------------------------------------------------------------ */
/* Envelope (implicit) gradients                                        */
/* ------------------------------------------------------------------ */
/* At the minimiser P* of the primal objective (entropic UOT, Section 2.1's
 * scaling loop run to its fixed point) the derivative of the optimal value
 * with respect to a parameter is the objective's partial derivative at
 * fixed P = P* (the P-derivative vanishes there):
 *   dL/dC_ij = P_ij,   dL/da_i = tau (1 - r_i/a_i),   dL/db_j = tau (1 - c_j/b_j)
 * (the KL terms' derivatives in their second argument; 0 when tau = inf).
 * Evaluated here at given scalings: P_ij = u_i K_ij v_j, r = P 1, c = P^T 1,
 * so it equals the gradient of the returned objective only as far as (u, v)
 * is a fixed point.  a_i, b_j > 0 required.  P may be NULL. */
ORC_EXPORT void orc_envelope_gradients(const double* K, const double* u, const double* v, const double* a,
                                       const double* b, int64_t n, int64_t m, double tau, double* grad_a,
                                       double* grad_b, double* P) {
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    orc_Kv(K, v, n, m, s);
    orc_KTu(K, u, n, m, w);
    for (int64_t i = 0; i < n; ++i) grad_a[i] = isinf(tau) ? 0.0 : tau * (1.0 - u[i] * s[i] / a[i]);
    for (int64_t j = 0; j < m; ++j) grad_b[j] = isinf(tau) ? 0.0 : tau * (1.0 - v[j] * w[j] / b[j]);
    if (P) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) P[i * m + j] = u[i] * K[i * m + j] * v[j];
    }
    free(s);
    free(w);
}

/* ------------------------------------------------------------------ */
/* Marginals and objective from potentials                              */
/* ------------------------------------------------------------------ */

/* Plan written through the potentials of its total scalings, f = eps log u,
 * g = eps log v:  P_ij = u_i K_ij v_j = exp((f_i + g_j - C_ij)/eps), finite
 * even where u, v overflow.  r = P 1 and c = P^T 1, each summed in
 * ascending index order.  f_i or g_j = -inf gives a zero row or column. */
ORC_EXPORT void orc_potential_marginals(const double* C, const double* f, const double* g,
                                        int64_t n, int64_t m, double eps, double* r, double* c) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) acc += exp((f[i] + g[j] - C[i * m + j]) / eps);
        r[i] = acc;
    }
    const int64_t BLK = 64;
    int64_t nblk = (m + BLK - 1) / BLK;
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t j0 = blk * BLK, j1 = j0 + BLK < m ? j0 + BLK : m;
        double acc[64];
        for (int64_t j = j0; j < j1; ++j) acc[j - j0] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j) acc[j - j0] += exp((f[i] + g[j] - C[i * m + j]) / eps);
        for (int64_t j = j0; j < j1; ++j) c[j] = acc[j - j0];
    }
}

/* The objective of orc_loss_identity with the log scalings given as
 * potentials (log u = f/eps, log v = g/eps):
 *   sum_i r_i f_i + sum_j c_j g_j - eps sum_i r_i + tau KL~(r|a) + tau KL~(c|b). */
ORC_EXPORT double orc_loss_potentials(const double* f, const double* g, const double* r,
                                      const double* c, const double* a, const double* b,
                                      int64_t n, int64_t m, double eps, double tau) {
    double sr = 0.0, sc = 0.0, mass = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (r[i] > 0.0) sr += r[i] * f[i];
        mass += r[i];
    }
    for (int64_t j = 0; j < m; ++j)
        if (c[j] > 0.0) sc += c[j] * g[j];
    double L = sr + sc - eps * mass;
    if (!isinf(tau)) {
        double kr = 0.0, kc = 0.0;
        for (int64_t i = 0; i < n; ++i) kr += orc_kl_term(r[i], a[i]);
        for (int64_t j = 0; j < m; ++j) kc += orc_kl_term(c[j], b[j]);
        L += tau * (kr + kc);
    }
    return L;
}

/* ------------------------------------------------------------------ */
/* Low-precision storage of the kernel                                  */
/* ------------------------------------------------------------------ */

/*
 * Value that a non-negative FP64 number takes once stored in a narrow
 * format, returned as FP64 (kind 1: bfloat16, kind 2: OCP E4M3FN, kind 3:
 * binary32 through the C conversion).  All round to nearest with ties to
 * even; the first two are written from the format definitions:
 *   bfloat16: 8 significant bits, exponent range of binary32; values below
 *             the smallest normal 2^-126 are stored as 0 (no subnormals);
 *   E4M3FN:   4 exponent bits (bias 7) and 3 fraction bits; normal values
 *             (1 + k/8) 2^e for e = -6 .. 8, subnormals k 2^-9 (k = 0 .. 7),
 *             largest finite 448; anything larger saturates to 448.
 * x = m 2^e with m in [1, 2): the stored value is rint(m 2^(p-1)) 2^(e-p+1)
 * with p significant bits (rint rounds ties to even in the default mode).
 */
ORC_EXPORT void orc_round_storage(const double* x, int64_t count, int kind, double* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        double xv = x[t];
        double r;
        if (!(xv > 0.0)) {
            r = 0.0;
        } else if (kind == 3) {
            r = (double)(float)xv;
        } else if (kind == 1) {
            if (xv < ldexp(1.0, -126)) {
                r = 0.0;
            } else {
                int e2;
                double mfr = frexp(xv, &e2);            /* xv = mfr 2^e2, mfr in [0.5, 1) */
                r = ldexp(rint(ldexp(mfr, 8)), e2 - 8);  /* 8 significant bits */
            }
        } else {
            if (xv >= 448.0) {
                r = 448.0;
            } else if (xv < ldexp(1.0, -6)) {
                r = ldexp(rint(ldexp(xv, 9)), -9);      /* subnormal grid k 2^-9 */
            } else {
                int e2;
                double mfr = frexp(xv, &e2);
                r = ldexp(rint(ldexp(mfr, 4)), e2 - 4);  /* 4 significant bits */
                if (r > 448.0) r = 448.0;
            }
        }
        out[t] = r;
    }
}

/*
 * Absorbed iteration with a normalised, optionally low-precision kernel.
 *
 * Same iterates as orc_sinkhorn_stabilized on (f, g, u, v), with two
 * differences that define how a kernel of limited range and precision is
 * kept usable:
 *   - normalisation: whenever the kernel is (re)built, the potentials are
 *     first set to   f_i = min_j (C_ij - g_j),   then   g_j = min_i (C_ij - f_i),
 *     so every exponent (f_i + g_j - C_ij)/eps is <= 0 and every row and
 *     every column of Kt reaches exactly 1; u and v are rescaled so that the
 *     totals u e^{f/eps} and v e^{g/eps} do not change;
 *   - storage: Kt is held as the value its entries take in the stored
 *     format (kind 0: FP64 itself; 1: bfloat16; 2: E4M3FN of store_scale*Kt,
 *     divided back by store_scale; 3: binary32), see orc_round_storage.
 * Start: u = v = 1, f = g = 0, then normalise.  After iteration t (t =
 * check_every, 2 check_every, ... and t < max_iter) the largest of
 * |log u_i|, |log v_j| (over positive entries) is compared with a level,
 * initially the threshold; above it, v is absorbed (g += eps log v, v = 1)
 * and the kernel is normalised and rebuilt (u does not need absorbing: the
 * next half-step recomputes it against the new f).  The normalisation puts
 * part of the scalings back (what a kernel whose rows and columns all peak
 * at 1 cannot carry); the largest |log| right after the rebuild (that
 * residue) sets the next level: the threshold, or when the residue exceeds
 * it the residue plus half the threshold, at most 60 (unless the threshold
 * is larger), so a residue that absorption cannot remove does not trigger a
 * rebuild at every check.
 * Outputs: f_tot, g_tot = f + eps log u, g + eps log v (-inf where the
 * scaling is 0); r = u * (Kt v), c = v * (Kt^T u) for the final scalings
 * (the plan's marginals, with the stored kernel); *loss the objective from
 * those (the identity form of orc_loss_identity on log scalings);
 * *absorptions the count; checks and arms (optional, length max_iter) the
 * compared maximum and the level at each check (0 elsewhere).  Returns
 * iterations.
 */
ORC_EXPORT int64_t orc_sinkhorn_absorbed(const double* C, const double* a, const double* b,
                                         int64_t n, int64_t m, double eps, double tau,
                                         int64_t max_iter, double threshold, int64_t check_every,
                                         int kind, double store_scale,
                                         double* f_tot, double* g_tot, double* r, double* c,
                                         double* loss, int64_t* absorptions, double* checks,
                                         double* arms) {
    double fi = orc_fi(eps, tau);
    double* Kt = (double*)malloc(sizeof(double) * (size_t)(n * m));
    double* f = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)m);
    double* u = (double*)malloc(sizeof(double) * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * (size_t)m);
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t i = 0; i < n; ++i) { f[i] = 0.0; u[i] = 1.0; }
    for (int64_t j = 0; j < m; ++j) { g[j] = 0.0; v[j] = 1.0; }
    if (checks) for (int64_t t = 0; t < max_iter; ++t) checks[t] = 0.0;
    if (arms) for (int64_t t = 0; t < max_iter; ++t) arms[t] = 0.0;
    int64_t nabs = 0;
    double arm = threshold;      /* level a check compares against */
    for (int64_t t = 0; t <= max_iter; ++t) {
        int rebuild = (t == 0);
        if (t > 0 && threshold > 0.0 && t % check_every == 0 && t < max_iter) {
            double mx = 0.0;
            for (int64_t i = 0; i < n; ++i) if (u[i] > 0.0 && fabs(log(u[i])) > mx) mx = fabs(log(u[i]));
            for (int64_t j = 0; j < m; ++j) if (v[j] > 0.0 && fabs(log(v[j])) > mx) mx = fabs(log(v[j]));
            if (checks) checks[t - 1] = mx;
            if (arms) arms[t - 1] = arm;
            if (mx > arm) {
                for (int64_t j = 0; j < m; ++j) if (v[j] > 0.0) { g[j] += eps * log(v[j]); v[j] = 1.0; }
                rebuild = 2;
                ++nabs;
            }
        }
        if (rebuild) {
            /* normalise: new f from the current g, then new g from the new f */
            for (int64_t i = 0; i < n; ++i) {
                double mn = INFINITY;
                for (int64_t j = 0; j < m; ++j) if (C[i * m + j] - g[j] < mn) mn = C[i * m + j] - g[j];
                if (u[i] > 0.0) u[i] = exp(log(u[i]) + (f[i] - mn) / eps);
                f[i] = mn;
            }
            for (int64_t j = 0; j < m; ++j) {
                double mn = INFINITY;
                for (int64_t i = 0; i < n; ++i) if (C[i * m + j] - f[i] < mn) mn = C[i * m + j] - f[i];
                if (v[j] > 0.0) v[j] = exp(log(v[j]) + (g[j] - mn) / eps);
                g[j] = mn;
            }
            if (rebuild == 2) {
                double res = 0.0;
                for (int64_t i = 0; i < n; ++i) if (u[i] > 0.0 && fabs(log(u[i])) > res) res = fabs(log(u[i]));
                for (int64_t j = 0; j < m; ++j) if (v[j] > 0.0 && fabs(log(v[j])) > res) res = fabs(log(v[j]));
                if (!(res > threshold)) {
                    arm = threshold;
                } else {
                    arm = res + 0.5 * threshold < 60.0 ? res + 0.5 * threshold : 60.0;
                    if (arm < threshold) arm = threshold;
                }
            }
            orc_kernel(C, n, m, eps, f, g, Kt);
            if (kind == 1 || kind == 3) {
                orc_round_storage(Kt, n * m, kind, Kt);
            } else if (kind == 2) {
                for (int64_t k = 0; k < n * m; ++k) Kt[k] *= store_scale;
                orc_round_storage(Kt, n * m, 2, Kt);
                for (int64_t k = 0; k < n * m; ++k) Kt[k] /= store_scale;
            }
        }
        if (t == max_iter) break;
        orc_Kv(Kt, v, n, m, s);
        for (int64_t i = 0; i < n; ++i)
            u[i] = (a[i] == 0.0) ? 0.0 : pow(a[i] / s[i], fi) * exp(-(1.0 - fi) * f[i] / eps);
        orc_KTu(Kt, u, n, m, w);
        for (int64_t j = 0; j < m; ++j)
            v[j] = (b[j] == 0.0) ? 0.0 : pow(b[j] / w[j], fi) * exp(-(1.0 - fi) * g[j] / eps);
    }
    orc_Kv(Kt, v, n, m, s);
    orc_KTu(Kt, u, n, m, w);
    double sr = 0.0, sc = 0.0, mass = 0.0, kr = 0.0, kc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        r[i] = u[i] * s[i];
        f_tot[i] = (u[i] > 0.0) ? f[i] + eps * log(u[i]) : -INFINITY;
        if (r[i] > 0.0) sr += r[i] * (f_tot[i] / eps);
        mass += r[i];
    }
    for (int64_t j = 0; j < m; ++j) {
        c[j] = v[j] * w[j];
        g_tot[j] = (v[j] > 0.0) ? g[j] + eps * log(v[j]) : -INFINITY;
        if (c[j] > 0.0) sc += c[j] * (g_tot[j] / eps);
    }
    double L = eps * (sr + sc - mass);
    if (!isinf(tau)) {
        for (int64_t i = 0; i < n; ++i) kr += orc_kl_term(r[i], a[i]);
        for (int64_t j = 0; j < m; ++j) kc += orc_kl_term(c[j], b[j]);
        L += tau * (kr + kc);
    }
    *loss = L;
    if (absorptions) *absorptions = nabs;
    free(Kt); free(f); free(g); free(u); free(v); free(s); free(w);
    return max_iter;
}

/* ------------------------------------------------------------------ */
/* Log-domain (log-sum-exp) iteration and eps-scaling                   */
/* ------------------------------------------------------------------ */

/* LSE over a row of z_j = (g_j - C_ij) / eps (or a column of
 * (f_i - C_ij) / eps): M + log sum exp(z - M) with M = max z, so every
 * exponential is <= 1 whatever eps.  All z = -inf gives -inf. */
static double orc_lse_row(const double* Crow, const double* g, int64_t m, double eps) {
    double M = -INFINITY;
    for (int64_t j = 0; j < m; ++j) {
        double z = (g[j] - Crow[j]) / eps;
        if (z > M) M = z;
    }
    if (M == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) s += exp((g[j] - Crow[j]) / eps - M);
    return M + log(s);
}

/* Column LSEs L_j = LSE_i (f_i - C_ij) / eps for all j (column blocks). */
static void orc_lse_cols(const double* C, const double* f, int64_t n, int64_t m, double eps, double* L) {
    const int64_t BLK = 64;
    int64_t nblk = (m + BLK - 1) / BLK;
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t j0 = blk * BLK, j1 = j0 + BLK < m ? j0 + BLK : m;
        double M[64], s[64];
        for (int64_t j = j0; j < j1; ++j) M[j - j0] = -INFINITY;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j) {
                double z = (f[i] - C[i * m + j]) / eps;
                if (z > M[j - j0]) M[j - j0] = z;
            }
        for (int64_t j = j0; j < j1; ++j) s[j - j0] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j)
                if (M[j - j0] > -INFINITY) s[j - j0] += exp((f[i] - C[i * m + j]) / eps - M[j - j0]);
        for (int64_t j = j0; j < j1; ++j) L[j] = M[j - j0] == -INFINITY ? -INFINITY : M[j - j0] + log(s[j - j0]);
    }
}

/* Potential update fi (eps log target - eps L); zero mass gives -inf. */
static double orc_lse_update(double target, double L, double eps, double fi) {
    if (target == 0.0) return -INFINITY;
    return fi * (eps * log(target) - eps * L);
}

/*
 * The iteration of Section 2.1 (vector form, rows first) written on the
 * potentials f = eps log u, g = eps log v:
 *     f_i = fi (eps log a_i - eps LSE_j((g_j - C_ij)/eps))
 *     g_j = fi (eps log b_j - eps LSE_i((f_i - C_ij)/eps)),
 * from g = 0 (v = 1); in exact arithmetic the same iterates as
 * orc_sinkhorn on K = exp(-C/eps), at any eps (no exponential exceeds 1).
 *
 * eps-scaling (the paper gives no schedule; this is the reading used):
 * when eps0 > eps, stage k = 0, 1, ... runs at eps_k = max(eps, eps0 *
 * factor^k) (0 < factor < 1); every stage before the one at eps runs
 * stage_iters iterations, each starting from the previous stage's
 * potentials; the stage at eps runs up to max_iter iterations with the
 * stopping rule of orc_sinkhorn (relative L1 change of the column marginal
 * c_j = exp(g_j/eps + LSE_i((f_i - C_ij)/eps)), c_0 = 0 at the stage's
 * start).  Without scaling (eps0 <= eps) only that last stage runs.
 *
 * Outputs: f, g; r, c, the marginals of P_ij = exp((f_i + g_j - C_ij)/eps)
 * at the final potentials; *loss the objective (orc_loss_potentials);
 * *err the last error.  Returns the iterations run over all stages.
 */
ORC_EXPORT int64_t orc_sinkhorn_lse(const double* C, const double* a, const double* b,
                                    int64_t n, int64_t m, double eps, double tau,
                                    int64_t max_iter, double tol,
                                    double eps0, double factor, int64_t stage_iters,
                                    double* f, double* g, double* r, double* c,
                                    double* loss, double* err_out) {
    double* L = (double*)malloc(sizeof(double) * (size_t)m);
    double* c_prev = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t i = 0; i < n; ++i) f[i] = 0.0;
    for (int64_t j = 0; j < m; ++j) g[j] = 0.0;
    int64_t total = 0;
    double err = 0.0;
    double e = eps0 > eps ? eps0 : eps;
    for (;;) {
        const int last = !(e > eps);
        const double fi = orc_fi(e, tau);
        const int64_t T = last ? max_iter : stage_iters;
        for (int64_t j = 0; j < m; ++j) c_prev[j] = 0.0;
        for (int64_t t = 0; t < T; ++t) {
            #pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) f[i] = orc_lse_update(a[i], orc_lse_row(C + i * m, g, m, e), e, fi);
            orc_lse_cols(C, f, n, m, e, L);
            for (int64_t j = 0; j < m; ++j) g[j] = orc_lse_update(b[j], L[j], e, fi);
            ++total;
            if (last) {
                double num = 0.0, den = 0.0;
                for (int64_t j = 0; j < m; ++j) {
                    double cj = exp(g[j] / e + L[j]);
                    num += fabs(cj - c_prev[j]);
                    den += fabs(cj);
                    c_prev[j] = cj;
                }
                err = num / den;
                if (tol > 0.0 && err <= tol) break;
            }
        }
        if (last) break;
        e = e * factor > eps ? e * factor : eps;
    }
    /* marginals at the final potentials */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = exp(f[i] / eps + orc_lse_row(C + i * m, g, m, eps));
    orc_lse_cols(C, f, n, m, eps, L);
    for (int64_t j = 0; j < m; ++j) c[j] = exp(g[j] / eps + L[j]);
    *loss = orc_loss_potentials(f, g, r, c, a, b, n, m, eps, tau);
    if (err_out) *err_out = err;
    free(L);
    free(c_prev);
    return total;
}
