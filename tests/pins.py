"""Independent mathematics that pins the FP64 oracle (and, at full size, the
HIP path) without running either of them.

Nothing here calls the oracle or the HIP library.  Each function derives a
value from the problem statement of Section 2.1 (rows and columns rescaled
alternately with factor (target / sum)^fi, fi = tau/(tau+eps), written on
scaling vectors) by a different route than the solver takes:

* ``one_by_one``     -- 1 x 1 problem: the iteration is linear in logs.
* ``rank1``          -- separable cost C_ij = alpha_i + beta_j: the iterates
                        depend on one scalar sigma_t = k2 . v_t whose log obeys
                        a linear recurrence, solved in closed form.
* ``newton_dual``    -- damped Newton on the concave dual of the entropic UOT
                        problem (brute force for tiny sizes).
* ``paper_matrix_form`` -- the paper's literal in-place row/column rescaling of
                        the matrix (Section 2.1, Algorithm 1's order of work
                        but rows first), used for the balanced (fi = 1) check.
* ``dual_value``     -- the dual objective D(f, g), for monotone ascent.
"""
from __future__ import annotations

import math

import numpy as np


def fi_of(eps: float, tau: float) -> float:
    return 1.0 if math.isinf(tau) else tau / (tau + eps)


# ---------------------------------------------------------------------------
# 1 x 1 closed form
# ---------------------------------------------------------------------------

def one_by_one(a: float, b: float, C: float, eps: float, tau: float, T: int):
    """Iterates (u_T, v_T) of the 1 x 1 problem from v_0 = 1.

    With l = log: l u_t = fi (l a - l k - l v_{t-1}), l v_t = fi (l b - l k - l u_t),
    l k = -C/eps.  Unrolled as a sum of a geometric series."""
    fi = fi_of(eps, tau)
    lk = -C / eps
    la, lb = math.log(a), math.log(b)
    # l v_t = fi (lb - lk) - fi^2 (la - lk) + fi^2 l v_{t-1}  => affine recurrence
    alpha = fi * (lb - lk) - fi * fi * (la - lk)
    q = fi * fi
    if T == 0:
        return 1.0, 1.0
    # l v_{T-1} in closed form (l v_0 = 0)
    if q == 1.0:
        lv_prev = alpha * (T - 1)
    else:
        lv_prev = alpha * (1.0 - q ** (T - 1)) / (1.0 - q)
    lu = fi * (la - lk - lv_prev)
    lv = fi * (lb - lk - lu)
    return math.exp(lu), math.exp(lv)


def one_by_one_log(a: float, b: float, C: float, eps: float, tau: float, T: int):
    """(log u_T, log v_T) of the 1 x 1 problem from v_0 = 1, the recurrence
    of one_by_one kept in logs (finite where u, v leave the FP64 range)."""
    fi = fi_of(eps, tau)
    lk = -C / eps
    la, lb = math.log(a), math.log(b)
    alpha = fi * (lb - lk) - fi * fi * (la - lk)
    q = fi * fi
    if T == 0:
        return 0.0, 0.0
    lv_prev = alpha * (T - 1) if q == 1.0 else alpha * (1.0 - q ** (T - 1)) / (1.0 - q)
    lu = fi * (la - lk - lv_prev)
    lv = fi * (lb - lk - lu)
    return lu, lv


def one_by_one_limit(a: float, b: float, C: float, eps: float, tau: float) -> float:
    """Optimal plan of the 1 x 1 problem: exp((tau (log a + log b) - C) / (eps + 2 tau))."""
    return math.exp((tau * (math.log(a) + math.log(b)) - C) / (eps + 2.0 * tau))


# ---------------------------------------------------------------------------
# Rank-1 (separable) cost closed form
# ---------------------------------------------------------------------------

def _logsumexp(z: np.ndarray) -> float:
    mx = float(np.max(z))
    return mx + math.log(float(np.sum(np.exp(z - mx))))


def rank1(alpha, beta, a, b, eps: float, tau: float, T: int):
    """(log u_T, log v_T) for C_ij = alpha_i + beta_j from v_0 = 1.

    K = k1 k2^T with k1 = e^{-alpha/eps}, k2 = e^{-beta/eps}.  With
    sigma_t = k2 . v_t: u_t = (a / (k1 sigma_{t-1}))^fi, k1 . u_t = A sigma_{t-1}^{-fi},
    v_t = (b / (k2 A sigma_{t-1}^{-fi}))^fi, hence
    log sigma_t = log B - fi log A + fi^2 log sigma_{t-1},
    A = sum k1^{1-fi} a^fi, B = sum k2^{1-fi} b^fi.  Entries with zero mass
    are not supported."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    fi = fi_of(eps, tau)
    lk1 = -alpha / eps
    lk2 = -beta / eps
    la, lb = np.log(a), np.log(b)
    logA = _logsumexp((1.0 - fi) * lk1 + fi * la)
    logB = _logsumexp((1.0 - fi) * lk2 + fi * lb)
    lsig0 = _logsumexp(lk2)
    c0 = logB - fi * logA
    q = fi * fi
    if T == 0:
        return np.zeros_like(a), np.zeros_like(b)
    n_steps = T - 1
    if q == 1.0:
        lsig = lsig0 + n_steps * c0
    else:
        lsig = (q ** n_steps) * lsig0 + c0 * (1.0 - q ** n_steps) / (1.0 - q)
    lu = fi * (la - lk1 - lsig)
    lv = fi * (lb - lk2 - logA + fi * lsig)
    return lu, lv


# ---------------------------------------------------------------------------
# Dual objective and Newton solve (tiny sizes)
# ---------------------------------------------------------------------------

def dual_value(f, g, C, a, b, eps: float, tau: float) -> float:
    """D(f,g) = -tau sum a (e^{-f/tau} - 1) - tau sum b (e^{-g/tau} - 1)
                - eps sum_ij exp((f_i + g_j - C_ij)/eps)."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    P = np.exp((f[:, None] + g[None, :] - C) / eps)
    return float(-tau * np.sum(a * np.expm1(-f / tau)) - tau * np.sum(b * np.expm1(-g / tau))
                 - eps * np.sum(P))


def newton_dual(C, a, b, eps: float, tau: float, tol: float = 1e-14, max_steps: int = 200):
    """Maximise the (strictly concave, tau < inf) dual by damped Newton.

    Returns (u, v) = (e^{f/eps}, e^{g/eps}) at the optimum, and the final
    gradient norm."""
    C = np.asarray(C, dtype=np.float64)
    n, m = C.shape
    f = np.zeros(n)
    g = np.zeros(m)

    def grad_hess(f, g):
        P = np.exp((f[:, None] + g[None, :] - C) / eps)
        ea = a * np.exp(-f / tau)
        eb = b * np.exp(-g / tau)
        gf = ea - P.sum(axis=1)
        gg = eb - P.sum(axis=0)
        H = np.zeros((n + m, n + m))
        H[:n, :n] = np.diag(-ea / tau - P.sum(axis=1) / eps)
        H[n:, n:] = np.diag(-eb / tau - P.sum(axis=0) / eps)
        H[:n, n:] = -P / eps
        H[n:, :n] = -P.T / eps
        return np.concatenate([gf, gg]), H

    gnorm = np.inf
    for _ in range(max_steps):
        gr, H = grad_hess(f, g)
        gnorm = float(np.max(np.abs(gr)))
        if gnorm < tol:
            break
        step = np.linalg.solve(H, -gr)
        D0 = dual_value(f, g, C, a, b, eps, tau)
        t = 1.0
        while t > 1e-12:
            fn = f + t * step[:n]
            gn = g + t * step[n:]
            if dual_value(fn, gn, C, a, b, eps, tau) >= D0 + 1e-4 * t * float(gr @ step):
                break
            t *= 0.5
        f, g = fn, gn
    return np.exp(f / eps), np.exp(g / eps), gnorm


# ---------------------------------------------------------------------------
# The paper's literal matrix-rescaling form
# ---------------------------------------------------------------------------

def paper_matrix_form(K, a, b, eps: float, tau: float, T: int) -> np.ndarray:
    """Rescale a copy of K in place, rows then columns, T times, with factors
    (target / current sum)^fi (Section 2.1).  Returns the rescaled matrix."""
    A = np.array(K, dtype=np.float64, copy=True)
    fi = fi_of(eps, tau)
    for _ in range(T):
        rs = A.sum(axis=1)
        alpha = np.where(a > 0, (a / np.where(rs > 0, rs, 1.0)) ** fi, 0.0)
        A *= alpha[:, None]
        cs = A.sum(axis=0)
        beta = np.where(b > 0, (b / np.where(cs > 0, cs, 1.0)) ** fi, 0.0)
        A *= beta[None, :]
    return A


def primal_value(P, C, a, b, eps: float, tau: float) -> float:
    """<C,P> + eps sum P(log P - 1) + tau KL~(P1|a) + tau KL~(P^T1|b), written
    with NumPy (a second, independent transcription of the definition)."""
    P = np.asarray(P, dtype=np.float64)
    r = P.sum(axis=1)
    c = P.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        ent = np.where(P > 0, P * (np.log(P) - 1.0), 0.0).sum()
        val = float((C * P).sum() + eps * ent)
        if not math.isinf(tau):
            kr = np.where(r > 0, r * np.log(r / a), 0.0).sum() - r.sum() + a.sum()
            kc = np.where(c > 0, c * np.log(c / b), 0.0).sum() - c.sum() + b.sum()
            val += tau * float(kr + kc)
    return val
