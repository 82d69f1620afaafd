"""FP64 CPU oracle for the UOT Sinkhorn loop -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``uot_oracle.c`` (plain C,
FP64, OpenMP across independent rows) with NumPy arrays and shares no code
with the HIP library.

Functions follow the paper's Section 2.1 problem statement written on
scaling vectors (the reading used throughout: rows first from v = 1, the
exponent fi = tau/(tau+eps)).  Where the paper is silent the readings are
stated in ``uot_oracle.c``'s header.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uot_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile ``uot_oracle.c`` into ``liboracle.so`` with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_cost_points.argtypes = [_dp, _dp, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_cost_points.restype = None
        lib.orc_kernel.argtypes = [_dp, _i64, _i64, ctypes.c_double, _dp, _dp, _dp]
        lib.orc_kernel.restype = None
        lib.orc_sinkhorn.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double, ctypes.c_double,
                                     _i64, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _dp]
        lib.orc_sinkhorn.restype = _i64
        lib.orc_loss_direct.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _i64, _i64,
                                        ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_loss_direct.restype = ctypes.c_double
        lib.orc_loss_identity.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _i64, _i64,
                                          ctypes.c_double, ctypes.c_double]
        lib.orc_loss_identity.restype = ctypes.c_double
        lib.orc_sinkhorn_stabilized.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double,
                                                ctypes.c_double, _i64, ctypes.c_double, _dp, _dp,
                                                ctypes.POINTER(_i64)]
        lib.orc_sinkhorn_stabilized.restype = _i64
        lib.orc_adjoint.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double, ctypes.c_double,
                                    _i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_adjoint.restype = None
        lib.orc_grad_points_sqeuclid.argtypes = [_dp, _dp, _dp, _i64, _i64, _i64, _dp]
        lib.orc_grad_points_sqeuclid.restype = None
        lib.orc_round_storage.argtypes = [_dp, _i64, ctypes.c_int, _dp]
        lib.orc_round_storage.restype = None
        lib.orc_sinkhorn_absorbed.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double,
                                              ctypes.c_double, _i64, ctypes.c_double, _i64,
                                              ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp,
                                              _dp, ctypes.POINTER(_i64), _dp, _dp]
        lib.orc_sinkhorn_absorbed.restype = _i64
        lib.orc_matrix_rescale.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double, ctypes.c_double, _i64, _dp,
                                           _dp]
        lib.orc_matrix_rescale.restype = None
        lib.orc_envelope_gradients.argtypes = [_dp, _dp, _dp, _dp, _dp, _i64, _i64, ctypes.c_double, _dp, _dp,
                                               _dp]
        lib.orc_envelope_gradients.restype = None
        lib.orc_grad_target_sqeuclid.argtypes = [_dp, _dp, _dp, _i64, _i64, _i64, _dp]
        lib.orc_grad_target_sqeuclid.restype = None
        lib.orc_potential_marginals.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double, _dp, _dp]
        lib.orc_potential_marginals.restype = None
        lib.orc_loss_potentials.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _i64, _i64, ctypes.c_double,
                                            ctypes.c_double]
        lib.orc_loss_potentials.restype = ctypes.c_double
        lib.orc_sinkhorn_lse.argtypes = [_dp, _dp, _dp, _i64, _i64, ctypes.c_double, ctypes.c_double, _i64,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, _i64, _dp, _dp, _dp,
                                         _dp, _dp, _dp]
        lib.orc_sinkhorn_lse.restype = _i64
        _lib = lib
    return _lib


def _p(arr: Optional[np.ndarray]):
    if arr is None:
        return None
    assert arr.dtype == np.float64 and arr.flags["C_CONTIGUOUS"], "oracle takes C-contiguous float64"
    return arr.ctypes.data_as(_dp)


def _f64(arr) -> np.ndarray:
    return np.ascontiguousarray(arr, dtype=np.float64)


# ---------------------------------------------------------------------------
# Cost and kernel
# ---------------------------------------------------------------------------

def cost_points(x, y, kind: int = 0, normalize: bool = False) -> np.ndarray:
    """Dense cost from points: squared Euclidean (kind 0) or 1 - x.y (kind 1)."""
    x = _f64(x)
    y = _f64(y)
    n, d = x.shape
    m = y.shape[0]
    C = np.empty((n, m), dtype=np.float64)
    _load().orc_cost_points(_p(x), _p(y), n, m, d, int(kind), int(bool(normalize)), _p(C))
    return C


def kernel(C, eps: float, f=None, g=None) -> np.ndarray:
    """Gibbs kernel exp((f_i + g_j - C_ij)/eps) (f = g = 0 by default)."""
    C = _f64(C)
    n, m = C.shape
    K = np.empty_like(C)
    _load().orc_kernel(_p(C), n, m, float(eps), _p(None if f is None else _f64(f)),
                       _p(None if g is None else _f64(g)), _p(K))
    return K


# ---------------------------------------------------------------------------
# Solver
# ---------------------------------------------------------------------------

@dataclass
class Result:
    u: np.ndarray
    v: np.ndarray
    r: np.ndarray          # row marginal u * (K v)
    c: np.ndarray          # column marginal v * (K^T u)
    iters: int
    err: float
    loss: float
    trace: Optional[dict] = None


def sinkhorn(K, a, b, eps: float, tau: float, max_iter: int, tol: float = 0.0,
             u0=None, v0=None, trace: bool = False) -> Result:
    """Plain FP64 UOT Sinkhorn in vector form, rows first, from v = 1."""
    K = _f64(K)
    a = _f64(a)
    b = _f64(b)
    n, m = K.shape
    assert a.shape == (n,) and b.shape == (m,)
    u = np.empty(n)
    v = np.empty(m)
    s_fin = np.empty(n)
    w_fin = np.empty(m)
    err = ctypes.c_double(0.0)
    tr = None
    if trace:
        T = max(int(max_iter), 0)
        tr = {"v": np.empty((T + 1, m)), "s": np.empty((max(T, 1), n)),
              "u": np.empty((max(T, 1), n)), "w": np.empty((max(T, 1), m))}
    it = _load().orc_sinkhorn(
        _p(K), _p(a), _p(b), n, m, float(eps), float(tau), int(max_iter), float(tol),
        _p(None if u0 is None else _f64(u0)), _p(None if v0 is None else _f64(v0)),
        _p(u), _p(v), _p(s_fin), _p(w_fin), ctypes.byref(err),
        _p(tr["v"]) if tr else None, _p(tr["s"]) if tr else None,
        _p(tr["u"]) if tr else None, _p(tr["w"]) if tr else None)
    r = u * s_fin
    c = v * w_fin
    loss = loss_identity(u, v, r, c, a, b, eps, tau)
    if tr is not None:
        tr["T"] = int(it)
    return Result(u=u, v=v, r=r, c=c, iters=int(it), err=float(err.value), loss=loss, trace=tr)


def loss_identity(u, v, r, c, a, b, eps: float, tau: float) -> float:
    """Objective from O(n+m) quantities (u, v, the marginals, a, b)."""
    u, v, r, c, a, b = map(_f64, (u, v, r, c, a, b))
    return float(_load().orc_loss_identity(_p(u), _p(v), _p(r), _p(c), _p(a), _p(b),
                                           u.shape[0], v.shape[0], float(eps), float(tau)))


def loss_direct(C, K, u, v, a, b, eps: float, tau: float):
    """Objective summed entry by entry over the plan; returns (loss, <C,P>)."""
    C, K, u, v, a, b = map(_f64, (C, K, u, v, a, b))
    tc = ctypes.c_double(0.0)
    L = _load().orc_loss_direct(_p(C), _p(K), _p(u), _p(v), _p(a), _p(b), u.shape[0],
                                v.shape[0], float(eps), float(tau), ctypes.byref(tc))
    return float(L), float(tc.value)


def sinkhorn_stabilized(C, a, b, eps: float, tau: float, max_iter: int, threshold: float):
    """Absorbed iteration; returns (f, g, absorptions) with total scalings e^{f/eps}, e^{g/eps}."""
    C = _f64(C)
    a = _f64(a)
    b = _f64(b)
    n, m = C.shape
    f = np.empty(n)
    g = np.empty(m)
    nabs = _i64(0)
    _load().orc_sinkhorn_stabilized(_p(C), _p(a), _p(b), n, m, float(eps), float(tau),
                                    int(max_iter), float(threshold), _p(f), _p(g),
                                    ctypes.byref(nabs))
    return f, g, int(nabs.value)


def adjoint(K, a, b, eps: float, tau: float, res: Result, want_G: bool = True):
    """Reverse-mode gradient through the unrolled iteration of ``res``.

    Returns (grad_a, grad_b, G) with G = dL/dC (None unless want_G)."""
    assert res.trace is not None, "run sinkhorn(..., trace=True) first"
    K = _f64(K)
    a = _f64(a)
    b = _f64(b)
    n, m = K.shape
    T = res.trace["T"]
    assert T >= 1
    ga = np.empty(n)
    gb = np.empty(m)
    G = np.empty((n, m)) if want_G else None
    tr = res.trace
    _load().orc_adjoint(_p(K), _p(a), _p(b), n, m, float(eps), float(tau), int(T),
                        _p(tr["v"]), _p(tr["s"]), _p(tr["u"]), _p(tr["w"]),
                        _p(ga), _p(gb), _p(G))
    return ga, gb, G


def matrix_rescale(A, a, b, eps: float, tau: float, T: int):
    """The paper's literal in-place rescaling of a copy of A (column factors
    first, then each row, T iterations); returns (A_T, r, c)."""
    A = np.array(A, dtype=np.float64, copy=True, order="C")
    a = _f64(a)
    b = _f64(b)
    n, m = A.shape
    r = np.empty(n)
    c = np.empty(m)
    _load().orc_matrix_rescale(_p(A), _p(a), _p(b), n, m, float(eps), float(tau), int(T), _p(r), _p(c))
    return A, r, c


def envelope_gradients(K, u, v, a, b, tau: float, want_P: bool = True):
    """Implicit (envelope) gradients at the scalings (u, v): returns
    (grad_a, grad_b, P) with dL/dC = P = diag(u) K diag(v) (None unless
    want_P), dL/da = tau (1 - r/a), dL/db = tau (1 - c/b)."""
    K, u, v, a, b = map(_f64, (K, u, v, a, b))
    n, m = K.shape
    ga = np.empty(n)
    gb = np.empty(m)
    P = np.empty((n, m)) if want_P else None
    _load().orc_envelope_gradients(_p(K), _p(u), _p(v), _p(a), _p(b), n, m, float(tau), _p(ga), _p(gb), _p(P))
    return ga, gb, P


def grad_points_sqeuclid(G, x, y) -> np.ndarray:
    """dL/dx_i = 2 sum_j G_ij (x_i - y_j) for an un-normalised squared-Euclidean cost."""
    G, x, y = map(_f64, (G, x, y))
    n, d = x.shape
    m = y.shape[0]
    gx = np.empty((n, d))
    _load().orc_grad_points_sqeuclid(_p(G), _p(x), _p(y), n, m, d, _p(gx))
    return gx


def grad_target_sqeuclid(G, x, y) -> np.ndarray:
    """dL/dy_j = 2 sum_i G_ij (y_j - x_i) for an un-normalised squared-Euclidean cost."""
    G, x, y = map(_f64, (G, x, y))
    n, d = x.shape
    m = y.shape[0]
    gy = np.empty((m, d))
    _load().orc_grad_target_sqeuclid(_p(G), _p(x), _p(y), n, m, d, _p(gy))
    return gy


def potential_marginals(C, f, g, eps: float):
    """Row and column sums of the plan exp((f_i + g_j - C_ij)/eps); returns (r, c)."""
    C, f, g = map(_f64, (C, f, g))
    n, m = C.shape
    r = np.empty(n)
    c = np.empty(m)
    _load().orc_potential_marginals(_p(C), _p(f), _p(g), n, m, float(eps), _p(r), _p(c))
    return r, c


def loss_potentials(f, g, r, c, a, b, eps: float, tau: float) -> float:
    """The objective from the potentials f = eps log u, g = eps log v and the marginals."""
    f, g, r, c, a, b = map(_f64, (f, g, r, c, a, b))
    return float(_load().orc_loss_potentials(_p(f), _p(g), _p(r), _p(c), _p(a), _p(b), f.shape[0],
                                             g.shape[0], float(eps), float(tau)))


_STORAGE_KINDS = {"bf16": 1, "e4m3": 2, "f32": 3}


def round_storage(x, kind: str) -> np.ndarray:
    """Values of non-negative ``x`` once stored as bfloat16 (``"bf16"``), OCP
    E4M3FN (``"e4m3"``) or binary32 (``"f32"``), round to nearest even,
    returned in FP64."""
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_round_storage(_p(x), x.size, _STORAGE_KINDS[kind], _p(out))
    return out


@dataclass
class AbsorbedResult:
    f: np.ndarray          # potentials of the total scalings: u_tot = e^{f/eps}
    g: np.ndarray
    r: np.ndarray          # row marginal with the stored kernel
    c: np.ndarray          # column marginal with the stored kernel
    loss: float
    absorptions: int
    checks: np.ndarray     # compared maximum |log| at each check (0 elsewhere)
    arms: np.ndarray       # level it was compared against (0 elsewhere)


def sinkhorn_absorbed(C, a, b, eps: float, tau: float, max_iter: int, threshold: float,
                      check_every: int = 1, storage: Optional[str] = None,
                      store_scale: float = 1.0) -> AbsorbedResult:
    """Absorbed iteration with row- and column-normalised kernel, optionally
    held in a narrow storage format (``None``, ``"f32"``, ``"bf16"`` or
    ``"e4m3"``); see orc_sinkhorn_absorbed for the absorption level."""
    C = _f64(C)
    a = _f64(a)
    b = _f64(b)
    n, m = C.shape
    f = np.empty(n)
    g = np.empty(m)
    r = np.empty(n)
    c = np.empty(m)
    loss = ctypes.c_double(0.0)
    nabs = _i64(0)
    checks = np.zeros(max(int(max_iter), 1))
    arms = np.zeros(max(int(max_iter), 1))
    kind = 0 if storage is None else _STORAGE_KINDS[storage]
    _load().orc_sinkhorn_absorbed(_p(C), _p(a), _p(b), n, m, float(eps), float(tau), int(max_iter),
                                  float(threshold), int(check_every), kind, float(store_scale),
                                  _p(f), _p(g), _p(r), _p(c), ctypes.byref(loss), ctypes.byref(nabs),
                                  _p(checks), _p(arms))
    return AbsorbedResult(f=f, g=g, r=r, c=c, loss=float(loss.value), absorptions=int(nabs.value),
                          checks=checks[:max_iter], arms=arms[:max_iter])


@dataclass
class LseResult:
    f: np.ndarray          # eps log u
    g: np.ndarray          # eps log v
    r: np.ndarray          # row marginal of P = exp((f_i + g_j - C_ij)/eps)
    c: np.ndarray          # column marginal
    loss: float
    iters: int             # iterations over all stages
    err: float


def sinkhorn_lse(C, a, b, eps: float, tau: float, max_iter: int, tol: float = 0.0,
                 eps0: float = 0.0, factor: float = 0.5, stage_iters: int = 0) -> LseResult:
    """Log-domain iteration on potentials (log-sum-exp rows and columns), with
    the eps-scaling schedule of orc_sinkhorn_lse when eps0 > eps."""
    C = _f64(C)
    a = _f64(a)
    b = _f64(b)
    n, m = C.shape
    f, g, r, c = np.empty(n), np.empty(m), np.empty(n), np.empty(m)
    loss = ctypes.c_double(0.0)
    err = ctypes.c_double(0.0)
    it = _load().orc_sinkhorn_lse(_p(C), _p(a), _p(b), n, m, float(eps), float(tau), int(max_iter), float(tol),
                                  float(eps0), float(factor), int(stage_iters), _p(f), _p(g), _p(r), _p(c),
                                  ctypes.byref(loss), ctypes.byref(err))
    return LseResult(f=f, g=g, r=r, c=c, loss=float(loss.value), iters=int(it), err=float(err.value))


def fi_exponent(eps: float, tau: float) -> float:
    """tau/(tau+eps); 1 in the balanced limit tau = inf."""
    return 1.0 if math.isinf(tau) else tau / (tau + eps)


def solve_problem(prob, max_iter: Optional[int] = None, tol: Optional[float] = None,
                  trace: bool = False):
    """Convenience: cost -> kernel -> Sinkhorn for a ``workloads.Problem``.

    Returns (Result, C, K)."""
    if prob.x is not None:
        C = cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    else:
        C = np.add.outer(_f64(prob.alpha), _f64(prob.beta))
    K = kernel(C, prob.eps)
    res = sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau,
                   prob.max_iter if max_iter is None else max_iter,
                   prob.tol if tol is None else tol, trace=trace)
    return res, C, K
