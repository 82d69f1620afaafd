"""MI355X (gfx950) entropic unbalanced-OT Sinkhorn: Python binding of libuot.so.

Every step of the solve runs in the HIP library; this module only marshals
torch device tensors (memory and streams) into the C-ABI of include/uot.h.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import (UOT_ACC_F32, UOT_ACC_F64, UOT_BF16, UOT_COST_COSINE, UOT_COST_SQEUCLID, UOT_F32, UOT_F64,
                   UOT_FLAG_NONFINITE, UOT_FLAG_NOT_CONVERGED, UOT_FLAG_ZERO_SUM, UOT_FP8_E4M3, UOTError)

__all__ = ["sinkhorn", "sinkhorn_backward", "sinkhorn_implicit_backward", "Gradients", "UOTLoss", "UOTCostLoss", "uot_loss", "uot_loss_cost", "cost_from_points", "kernel_from_cost",
           "kernel_to_f32", "matrix_rescale_", "MatrixResult", "sinkhorn_batched", "BatchedSolver", "BatchedResult", "plan", "sinkhorn_multi",
           "SinkhornResult", "UOTError", "lib_path",
           "UOT_F64", "UOT_F32", "UOT_BF16", "UOT_FP8_E4M3", "UOT_COST_SQEUCLID", "UOT_COST_COSINE"]

_DTYPES = {torch.float64: UOT_F64, torch.float32: UOT_F32, torch.bfloat16: UOT_BF16,
           torch.float8_e4m3fn: UOT_FP8_E4M3}
FP8_STORE_SCALE = 448.0   # an FP8 kernel from kernel_from_cost holds 448 * K
_ELEM = {UOT_F64: 8, UOT_F32: 4, UOT_BF16: 2, UOT_FP8_E4M3: 1}


def lib_path() -> str:
    return _lib.LIB_PATH


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _vec64(x: torch.Tensor, name: str, length: int, device) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if x.dtype != torch.float64 or x.dim() != 1 or x.shape[0] != length or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 vector of length {length}")
    return x


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def cost_from_points(x: torch.Tensor, y: torch.Tensor, kind: int = UOT_COST_SQEUCLID,
                     normalize_max: bool = False) -> torch.Tensor:
    """Dense FP64 cost (n x m) from FP64 points, computed by the library."""
    if x.dtype != torch.float64 or y.dtype != torch.float64:
        raise ValueError("points must be float64")
    x = x.contiguous()
    y = y.contiguous()
    n, d = x.shape
    m, d2 = y.shape
    if d != d2:
        raise ValueError("x and y must have the same dimension")
    L = _lib.lib()
    C = torch.empty((n, m), dtype=torch.float64, device=x.device)
    ws = _workspace(L.uot_cost_workspace_size(n, m), x.device)
    _lib.check(L.uot_cost_from_points(_ptr(x), _ptr(y), n, m, d, int(kind), int(bool(normalize_max)), _ptr(C), m,
                                      _ptr(ws), ws.numel(), _stream(x.device)))
    return C


def kernel_from_cost(C: torch.Tensor, eps: float, dtype: torch.dtype = torch.float32,
                     f: Optional[torch.Tensor] = None, g: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gibbs kernel exp((f_i + g_j - C_ij)/eps) rounded to ``dtype``.

    Returns an (n, ldk) tensor whose first m columns hold K (ldk = m rounded
    up to 64; padding columns are 0); use ``K[:, :m]`` for the logical view."""
    if C.dtype != torch.float64 or C.dim() != 2:
        raise ValueError("C must be a float64 matrix")
    if dtype not in _DTYPES:
        raise ValueError(f"unsupported K dtype {dtype}")
    n, m = C.shape
    ldk = (m + 63) // 64 * 64
    K = torch.empty((n, ldk), dtype=dtype, device=C.device)
    L = _lib.lib()
    _lib.check(L.uot_kernel_from_cost(_ptr(C), C.stride(0), n, m, float(eps), _ptr(f), _ptr(g), _DTYPES[dtype],
                                      _ptr(K), ldk, _stream(C.device)))
    return K


def kernel_to_f32(K: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
    """Decode a stored kernel (any supported dtype, contiguous, a multiple of
    16 bytes) to FP32 exactly as the streaming passes read it, times scale."""
    if K.dtype not in _DTYPES:
        raise ValueError(f"unsupported K dtype {K.dtype}")
    K = K.contiguous()
    out = torch.empty(K.shape, dtype=torch.float32, device=K.device)
    _lib.check(_lib.lib().uot_kernel_to_f32(_ptr(K), _DTYPES[K.dtype], K.numel(), float(scale), _ptr(out),
                                            _stream(K.device)))
    return out


@dataclass
class SinkhornResult:
    u: torch.Tensor
    v: torch.Tensor
    r: torch.Tensor
    c: torch.Tensor
    loss: torch.Tensor            # device FP64 scalar
    info_raw: torch.Tensor        # device bytes of uot_info
    profile: Optional[dict] = None
    f: Optional[torch.Tensor] = None    # eps log u (finite where u overflows)
    g: Optional[torch.Tensor] = None    # eps log v

    def info(self) -> dict:
        """Synchronises and decodes the device-resident report."""
        raw = bytes(self.info_raw.cpu().numpy().tobytes())
        inf = _lib.Info.from_buffer_copy(raw)
        return {"iters": int(inf.iters), "err": float(inf.err), "absorptions": int(inf.absorptions),
                "flags": int(inf.flags)}


def _problem(a, b, K, C, m_logical, eps, tau, device):
    n = a.shape[0]
    m = m_logical
    prob = _lib.Problem()
    prob.n = n
    prob.m = m
    prob.a = a.data_ptr()
    prob.b = b.data_ptr()
    if K is not None:
        if K.dtype not in _DTYPES:
            raise ValueError(f"unsupported K dtype {K.dtype}")
        if K.dim() != 2 or K.shape[0] != n or K.shape[1] < m or K.stride(1) != 1:
            raise ValueError("K must be an (n, ldk >= m) row-major matrix")
        ldk = K.stride(0)
        # The library reads whole 16-byte chunks: every row must own ldk elements.
        if K.storage_offset() + (n - 1) * ldk + ldk > K.untyped_storage().nbytes() // K.element_size():
            raise ValueError("K's storage must hold n * ldk elements")
        prob.k_dtype = _DTYPES[K.dtype]
        prob.K = K.data_ptr()
        prob.ldk = ldk
        prob.k_scale = 1.0 / FP8_STORE_SCALE if K.dtype == torch.float8_e4m3fn else 1.0
    else:
        prob.k_dtype = UOT_F32
        prob.K = None
        prob.ldk = 0
    if C is not None:
        if C.dtype != torch.float64 or C.shape[0] != n or C.shape[1] < m or C.stride(1) != 1:
            raise ValueError("C must be an (n, >= m) float64 row-major matrix")
        prob.C = C.data_ptr()
        prob.ldc = C.stride(0)
    prob.eps = float(eps)
    prob.tau = float(tau)
    return prob


def sinkhorn(a: torch.Tensor, b: torch.Tensor, K: Optional[torch.Tensor] = None, *, C: Optional[torch.Tensor] = None,
             m: Optional[int] = None, eps: float, tau: float, max_iter: int, tol: float = 0.0,
             fused: bool = True, accum: str = "f32", check_every: int = 1, tune: int = 0,
             k_dtype: Optional[torch.dtype] = None, u0: Optional[torch.Tensor] = None,
             v0: Optional[torch.Tensor] = None, persistent: bool = False,
             checkpoint_every: int = 0, absorb_log_threshold: float = 0.0,
             profile: bool = False, store_iterates: bool = False) -> SinkhornResult:
    """UOT Sinkhorn scaling loop on the GPU (see include/uot.h, uot_sinkhorn).

    ``K`` is an (n, ldk) FP32/FP64 kernel (as returned by kernel_from_cost);
    ``m`` is the logical column count (default ``b.shape[0]``).  Without K, the
    FP64 cost ``C`` is turned into a kernel of ``k_dtype`` inside the call.
    ``checkpoint_every=k`` keeps every k-th v for ``sinkhorn_backward``;
    ``store_iterates`` keeps every iterate instead ((2T + 1) m + 2T n
    doubles), so that the reverse pass repeats no forward pass."""
    device = a.device
    n = a.shape[0]
    m = b.shape[0] if m is None else int(m)
    a = _vec64(a, "a", n, device)
    b = _vec64(b, "b", m, device)
    prob = _problem(a, b, K, C, m, eps, tau, device)
    if K is None:
        if k_dtype is not None:
            prob.k_dtype = _DTYPES[k_dtype]
    opt = _lib.Options()
    opt.max_iter = int(max_iter)
    opt.check_every = int(check_every)
    opt.tol = float(tol)
    opt.fused = 1 if fused else 0
    opt.accum = UOT_ACC_F64 if accum == "f64" else UOT_ACC_F32
    opt.absorb_log_threshold = float(absorb_log_threshold)
    opt.checkpoint_every = int(checkpoint_every)
    opt.tune = int(tune)
    opt.u0 = None if u0 is None else _vec64(u0, "u0", n, device).data_ptr()
    opt.v0 = None if v0 is None else _vec64(v0, "v0", m, device).data_ptr()
    opt.persistent = 1 if persistent else 0
    opt.store_iterates = 1 if store_iterates else 0
    L = _lib.lib()
    need = L.uot_sinkhorn_workspace_size(ctypes.byref(prob), ctypes.byref(opt))
    if need == 0:
        _lib.check(L.uot_sinkhorn(ctypes.byref(prob), ctypes.byref(opt), None, None, 0, None))
    ws = _workspace(need, device)
    u = torch.empty(n, dtype=torch.float64, device=device)
    v = torch.empty(m, dtype=torch.float64, device=device)
    r = torch.empty(n, dtype=torch.float64, device=device)
    c = torch.empty(m, dtype=torch.float64, device=device)
    loss = torch.empty((), dtype=torch.float64, device=device)
    info = torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=device)
    ckpt = None
    if checkpoint_every > 0:
        slots = (int(max_iter) + int(checkpoint_every) - 1) // int(checkpoint_every) + 1
        ckpt = torch.zeros(slots * 2 * m, dtype=torch.float64, device=device)
    elif store_iterates and max_iter > 0:
        T = int(max_iter)
        ckpt = torch.empty((2 * T + 1) * m + 2 * T * n, dtype=torch.float64, device=device)
    fpot = torch.empty(n, dtype=torch.float64, device=device)
    gpot = torch.empty(m, dtype=torch.float64, device=device)
    out = _lib.Outputs(u.data_ptr(), v.data_ptr(), r.data_ptr(), c.data_ptr(), loss.data_ptr(), info.data_ptr(),
                       None if ckpt is None else ckpt.data_ptr(), fpot.data_ptr(), gpot.data_ptr())
    prof = None
    if profile:
        p = _lib.Profile()
        _lib.check(L.uot_sinkhorn_profiled(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(out), _ptr(ws),
                                           ws.numel(), _stream(device), ctypes.byref(p)))
        prof = {f: getattr(p, f) for f, _ in _lib.Profile._fields_}
    else:
        _lib.check(L.uot_sinkhorn(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(out), _ptr(ws), ws.numel(),
                                  _stream(device)))
    res = SinkhornResult(u=u, v=v, r=r, c=c, loss=loss, info_raw=info, profile=prof, f=fpot, g=gpot)
    res._keepalive = (ws, K, C, a, b)  # buffers must outlive the enqueued work
    res._problem = prob
    res._options = opt
    res.ckpt = ckpt
    return res


def sinkhorn_points(x: torch.Tensor, y: torch.Tensor, a: torch.Tensor, b: torch.Tensor, *, eps: float, tau: float,
                    max_iter: int, cost_scale: float = 1.0, tol: float = 0.0, check_every: int = 1,
                    u0: Optional[torch.Tensor] = None, v0: Optional[torch.Tensor] = None) -> SinkhornResult:
    """Kernel-free solve for the cost ``cost_scale * ||x_i - y_j||^2`` of 2-D
    or 3-D points (include/uot.h, uot_sinkhorn_points): K is recomputed in
    every pass, never stored."""
    device = a.device
    n, m = a.shape[0], b.shape[0]
    if x.dim() != 2 or y.dim() != 2 or x.shape[0] != n or y.shape[0] != m or x.shape[1] != y.shape[1]:
        raise ValueError("x must be (n, d) and y (m, d) with the lengths of a and b")
    dim = x.shape[1]
    x = x.to(device=device, dtype=torch.float64).contiguous()
    y = y.to(device=device, dtype=torch.float64).contiguous()
    a = _vec64(a, "a", n, device)
    b = _vec64(b, "b", m, device)
    prob = _problem(a, b, None, None, m, eps, tau, device)
    opt = _lib.Options()
    opt.max_iter = int(max_iter)
    opt.check_every = int(check_every)
    opt.tol = float(tol)
    opt.fused = 1
    opt.accum = UOT_ACC_F32
    opt.u0 = None if u0 is None else _vec64(u0, "u0", n, device).data_ptr()
    opt.v0 = None if v0 is None else _vec64(v0, "v0", m, device).data_ptr()
    L = _lib.lib()
    need = L.uot_sinkhorn_points_workspace_size(ctypes.byref(prob), dim, float(cost_scale), ctypes.byref(opt))
    if need == 0:
        _lib.check(L.uot_sinkhorn_points(ctypes.byref(prob), _ptr(x), _ptr(y), dim, float(cost_scale),
                                         ctypes.byref(opt), None, None, 0, None))
    ws = _workspace(need, device)
    u = torch.empty(n, dtype=torch.float64, device=device)
    v = torch.empty(m, dtype=torch.float64, device=device)
    r = torch.empty(n, dtype=torch.float64, device=device)
    c = torch.empty(m, dtype=torch.float64, device=device)
    loss = torch.empty((), dtype=torch.float64, device=device)
    info = torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=device)
    fpot = torch.empty(n, dtype=torch.float64, device=device)
    gpot = torch.empty(m, dtype=torch.float64, device=device)
    out = _lib.Outputs(u.data_ptr(), v.data_ptr(), r.data_ptr(), c.data_ptr(), loss.data_ptr(), info.data_ptr(),
                       None, fpot.data_ptr(), gpot.data_ptr())
    _lib.check(L.uot_sinkhorn_points(ctypes.byref(prob), _ptr(x), _ptr(y), dim, float(cost_scale),
                                     ctypes.byref(opt), ctypes.byref(out), _ptr(ws), ws.numel(), _stream(device)))
    res = SinkhornResult(u=u, v=v, r=r, c=c, loss=loss, info_raw=info, f=fpot, g=gpot)
    res._keepalive = (ws, x, y, a, b)
    return res


def sinkhorn_lse(C: torch.Tensor, a: torch.Tensor, b: torch.Tensor, *, eps: float, tau: float, max_iter: int,
                 m: Optional[int] = None, tol: float = 0.0, check_every: int = 1,
                 cost_dtype: torch.dtype = torch.float64, eps0: float = 0.0, factor: float = 0.5,
                 stage_iters: int = 0) -> SinkhornResult:
    """Log-domain solve on the FP64 cost ``C`` (include/uot.h,
    uot_sinkhorn_lse): potentials f, g, log-sum-exp passes reading C in
    ``cost_dtype`` (float64 or float32), optional eps-scaling from ``eps0``."""
    if C.dtype != torch.float64 or C.dim() != 2 or C.stride(1) != 1:
        raise ValueError("C must be a row-major float64 matrix")
    device = a.device
    n = a.shape[0]
    m = b.shape[0] if m is None else int(m)
    if C.stride(0) % 2:
        Cp = torch.zeros((C.shape[0], C.stride(0) + 1), dtype=torch.float64, device=device)
        Cp[:, :C.shape[1]] = C
        C = Cp
    a = _vec64(a, "a", n, device)
    b = _vec64(b, "b", m, device)
    prob = _problem(a, b, None, C, m, eps, tau, device)
    prob.k_dtype = _DTYPES[cost_dtype]
    opt = _lib.Options()
    opt.max_iter = int(max_iter)
    opt.check_every = int(check_every)
    opt.tol = float(tol)
    opt.fused = 1
    opt.accum = UOT_ACC_F32
    sch = _lib.EpsSchedule(float(eps0), float(factor), int(stage_iters), 0)
    L = _lib.lib()
    need = L.uot_sinkhorn_lse_workspace_size(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(sch))
    if need == 0:
        _lib.check(L.uot_sinkhorn_lse(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(sch), None, None, 0, None))
    ws = _workspace(need, device)
    u = torch.empty(n, dtype=torch.float64, device=device)
    v = torch.empty(m, dtype=torch.float64, device=device)
    r = torch.empty(n, dtype=torch.float64, device=device)
    c = torch.empty(m, dtype=torch.float64, device=device)
    loss = torch.empty((), dtype=torch.float64, device=device)
    info = torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=device)
    fpot = torch.empty(n, dtype=torch.float64, device=device)
    gpot = torch.empty(m, dtype=torch.float64, device=device)
    out = _lib.Outputs(u.data_ptr(), v.data_ptr(), r.data_ptr(), c.data_ptr(), loss.data_ptr(), info.data_ptr(),
                       None, fpot.data_ptr(), gpot.data_ptr())
    _lib.check(L.uot_sinkhorn_lse(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(sch), ctypes.byref(out),
                                  _ptr(ws), ws.numel(), _stream(device)))
    res = SinkhornResult(u=u, v=v, r=r, c=c, loss=loss, info_raw=info, f=fpot, g=gpot)
    res._keepalive = (ws, C, a, b)
    return res


@dataclass
class MatrixResult:
    alpha: torch.Tensor       # (n,) last row factors
    beta: torch.Tensor        # (m,) column factors of the next iteration
    r: torch.Tensor           # (n,) row sums of the rescaled matrix
    c: torch.Tensor           # (m,) column sums
    info_raw: torch.Tensor

    def info(self) -> dict:
        s = _lib.Info.from_buffer_copy(bytes(self.info_raw.cpu().numpy().tobytes()))
        return {"iters": s.iters, "err": s.err, "flags": s.flags}


def matrix_rescale_(A: torch.Tensor, a: torch.Tensor, b: torch.Tensor, *, m: Optional[int] = None, eps: float,
                    tau: float, max_iter: int, tol: float = 0.0, check_every: int = 1, tune: int = 0) -> MatrixResult:
    """The paper's literal in-place rescaling of ``A`` (include/uot.h,
    uot_matrix_rescale): ``A`` (n, ldk) FP32 or FP64 is modified in place."""
    if A.dtype not in (torch.float32, torch.float64):
        raise ValueError("A must be float32 or float64")
    device = A.device
    n = a.shape[0]
    m = b.shape[0] if m is None else int(m)
    a = _vec64(a, "a", n, device)
    b = _vec64(b, "b", m, device)
    prob = _problem(a, b, A, None, m, eps, tau, device)
    opt = _lib.Options()
    opt.max_iter = int(max_iter)
    opt.check_every = int(check_every)
    opt.tol = float(tol)
    opt.fused = 1
    opt.tune = int(tune)
    L = _lib.lib()
    need = L.uot_matrix_rescale_workspace_size(ctypes.byref(prob), ctypes.byref(opt))
    if need == 0:
        _lib.check(L.uot_matrix_rescale(ctypes.byref(prob), ctypes.byref(opt), None, None, 0, None))
    ws = _workspace(need, device)
    res = MatrixResult(alpha=torch.empty(n, dtype=torch.float64, device=device),
                       beta=torch.empty(m, dtype=torch.float64, device=device),
                       r=torch.empty(n, dtype=torch.float64, device=device),
                       c=torch.empty(m, dtype=torch.float64, device=device),
                       info_raw=torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=device))
    out = _lib.Outputs(res.alpha.data_ptr(), res.beta.data_ptr(), res.r.data_ptr(), res.c.data_ptr(), None,
                       res.info_raw.data_ptr(), None, None, None)
    _lib.check(L.uot_matrix_rescale(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(out), _ptr(ws), ws.numel(),
                                    _stream(device)))
    res._keep = (ws, a, b)
    return res


def plan(res: SinkhornResult, dtype: torch.dtype = torch.float64, from_cost: bool = False) -> torch.Tensor:
    """Dense plan of a solve (include/uot.h, uot_plan): u_i K_ij v_j from the
    solve's kernel, or (``from_cost``, needs the solve's C) the form
    exp((f_i + g_j - C_ij)/eps) from the potentials of the total scalings."""
    if dtype not in (torch.float64, torch.float32):
        raise ValueError("plan dtype must be float64 or float32")
    prob = res._problem
    n, m = res.u.shape[0], res.v.shape[0]
    P = torch.empty((n, m), dtype=dtype, device=res.u.device)
    p = _lib.Problem.from_buffer_copy(prob)
    L = _lib.lib()
    if from_cost:
        if not prob.C:
            raise ValueError("from_cost needs a solve given C")
        p.K = None
        args = (None, None, _ptr(res.f), _ptr(res.g))
    else:
        if not prob.K:
            raise ValueError("the solve built its kernel internally: use from_cost=True")
        args = (_ptr(res.u), _ptr(res.v), None, None)
    _lib.check(L.uot_plan(ctypes.byref(p), *args, _ptr(P), m, _DTYPES[dtype], _stream(res.u.device)))
    return P


@dataclass
class MultiResult:
    U: torch.Tensor           # (R, n) FP64
    V: torch.Tensor           # (R, m) FP64
    loss: torch.Tensor        # (R,) FP64
    info_raw: torch.Tensor

    def info(self) -> dict:
        s = _lib.Info.from_buffer_copy(bytes(self.info_raw.cpu().numpy().tobytes()))
        return {"iters": s.iters, "err": s.err, "absorptions": s.absorptions, "flags": s.flags}


def sinkhorn_multi(K: torch.Tensor, A: torch.Tensor, B: torch.Tensor, *, m: Optional[int] = None, eps: float,
                   tau: float, max_iter: int, tune: int = 0) -> MultiResult:
    """R histogram pairs sharing K (include/uot.h, uot_sinkhorn_multi).
    K: (n, ldk) FP32 or BF16; A: (R, n), B: (R, m) FP64, one histogram per row."""
    if K.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("K must be float32 or bfloat16")
    if A.dtype != torch.float64 or B.dtype != torch.float64 or A.dim() != 2 or B.dim() != 2:
        raise ValueError("A and B must be (R, n) and (R, m) float64 matrices")
    A = A.contiguous()
    B = B.contiguous()
    R, n = A.shape
    m = B.shape[1] if m is None else int(m)
    if B.shape != (R, m) or K.shape[0] != n or K.shape[1] < m or K.stride(1) != 1:
        raise ValueError("shapes of K, A and B do not match")
    device = K.device
    prob = _lib.Problem()
    prob.n, prob.m = n, m
    prob.k_dtype = _DTYPES[K.dtype]
    prob.K = K.data_ptr()
    prob.ldk = K.stride(0)
    prob.eps, prob.tau, prob.k_scale = float(eps), float(tau), 1.0
    opt = _lib.Options()
    opt.max_iter = int(max_iter)
    opt.check_every = 1
    opt.fused = 1
    opt.tune = int(tune)
    L = _lib.lib()
    need = L.uot_sinkhorn_multi_workspace_size(ctypes.byref(prob), R, ctypes.byref(opt))
    if need == 0:
        _lib.check(L.uot_sinkhorn_multi(ctypes.byref(prob), R, None, None, ctypes.byref(opt), None, None, None, None,
                                        None, 0, None))
    ws = _workspace(need, device)
    U = torch.empty((R, n), dtype=torch.float64, device=device)
    V = torch.empty((R, m), dtype=torch.float64, device=device)
    loss = torch.empty(R, dtype=torch.float64, device=device)
    info = torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=device)
    _lib.check(L.uot_sinkhorn_multi(ctypes.byref(prob), R, _ptr(A), _ptr(B), ctypes.byref(opt), _ptr(U), _ptr(V),
                                    _ptr(loss), _ptr(info), _ptr(ws), ws.numel(), _stream(device)))
    res = MultiResult(U, V, loss, info)
    res._keep = (ws, K, A, B)
    return res


@dataclass
class Gradients:
    """Outputs of sinkhorn_backward, each g times dL/d(input) or None."""
    grad_a: Optional[torch.Tensor] = None
    grad_b: Optional[torch.Tensor] = None
    grad_x: Optional[torch.Tensor] = None
    grad_C: Optional[torch.Tensor] = None
    grad_y: Optional[torch.Tensor] = None


def sinkhorn_backward(res: SinkhornResult, grad_loss: torch.Tensor, *, x: Optional[torch.Tensor] = None,
                      y: Optional[torch.Tensor] = None, want_a: bool = True, want_b: bool = True,
                      want_x: bool = True, want_C: bool = False, want_y: bool = False) -> Gradients:
    """Reverse pass of ``sinkhorn(..., checkpoint_every=k)`` or
    ``sinkhorn(..., store_iterates=True)`` (include/uot.h,
    uot_sinkhorn_backward).  ``grad_loss`` is a device FP64 scalar.  With the
    points ``x`` (n x d) and ``y`` (m x d) of an un-normalised squared-Euclidean
    cost, also dL/dx (``want_x``) and dL/dy (``want_y``); ``want_C`` gives
    the dense dL/dC (n x m FP64)."""
    if res.ckpt is None:
        raise ValueError("the forward call needs checkpoint_every > 0 or store_iterates")
    prob, opt = res._problem, res._options
    device = res.u.device
    n, m = res.u.shape[0], res.v.shape[0]
    g = grad_loss.reshape(()).to(dtype=torch.float64, device=device).contiguous()
    dim = 0
    if y is not None:
        if y.dtype != torch.float64 or y.dim() != 2 or y.shape[0] != m:
            raise ValueError("y must be an (m, d) float64 tensor")
        y = y.contiguous()
        dim = y.shape[1]
    if x is not None:
        if y is None or x.dtype != torch.float64 or x.shape != (n, dim):
            raise ValueError("x must be an (n, d) float64 tensor matching y")
        x = x.contiguous()
    if want_y and x is None:
        raise ValueError("want_y needs the points x and y")
    cost_grad = 1 if (want_C or want_y) else 0
    L = _lib.lib()
    need = L.uot_sinkhorn_backward_workspace_size(ctypes.byref(prob), ctypes.byref(opt), dim, cost_grad)
    if need == 0:
        _lib.check(L.uot_sinkhorn_backward(ctypes.byref(prob), ctypes.byref(opt), None, None, None, None, None,
                                           None, None, 0, None, None, dim, None, None, None, 0, None))
    ws = _workspace(need, device)
    out = Gradients()
    out.grad_a = torch.empty(n, dtype=torch.float64, device=device) if want_a else None
    out.grad_b = torch.empty(m, dtype=torch.float64, device=device) if want_b else None
    out.grad_x = torch.empty((n, dim), dtype=torch.float64, device=device) if (x is not None and want_x) else None
    out.grad_y = torch.empty((m, dim), dtype=torch.float64, device=device) if want_y else None
    out.grad_C = torch.empty((n, m), dtype=torch.float64, device=device) if want_C else None
    _lib.check(L.uot_sinkhorn_backward(ctypes.byref(prob), ctypes.byref(opt), _ptr(res.u), _ptr(res.v),
                                       _ptr(res.ckpt), _ptr(g), _ptr(out.grad_a), _ptr(out.grad_b),
                                       _ptr(out.grad_C), m, _ptr(x), _ptr(y), dim, _ptr(out.grad_x),
                                       _ptr(out.grad_y), _ptr(ws), ws.numel(), _stream(device)))
    out._keep = (ws, g, x, y)   # buffers must outlive the enqueued work
    return out


def sinkhorn_implicit_backward(res: SinkhornResult, grad_loss: torch.Tensor, *, x: Optional[torch.Tensor] = None,
                               y: Optional[torch.Tensor] = None, want_a: bool = True, want_b: bool = True,
                               want_x: bool = True, want_C: bool = False, want_y: bool = False) -> Gradients:
    """Implicit (envelope) gradients at the scalings of a converged
    ``sinkhorn`` call (include/uot.h, uot_sinkhorn_implicit_backward): no
    checkpoints, one marginal pass over K plus one per point coordinate."""
    prob, opt = res._problem, res._options
    device = res.u.device
    n, m = res.u.shape[0], res.v.shape[0]
    if opt.absorb_log_threshold > 0.0:
        raise ValueError("the implicit gradient needs the scalings of a solve without absorption")
    g = grad_loss.reshape(()).to(dtype=torch.float64, device=device).contiguous()
    dim = 0
    if y is not None:
        if y.dtype != torch.float64 or y.dim() != 2 or y.shape[0] != m:
            raise ValueError("y must be an (m, d) float64 tensor")
        y = y.contiguous()
        dim = y.shape[1]
    if x is not None:
        if y is None or x.dtype != torch.float64 or x.shape != (n, dim):
            raise ValueError("x must be an (n, d) float64 tensor matching y")
        x = x.contiguous()
    if (want_y or (want_x and x is not None)) and (x is None or y is None):
        raise ValueError("point gradients need x and y")
    L = _lib.lib()
    need = L.uot_sinkhorn_implicit_backward_workspace_size(ctypes.byref(prob), ctypes.byref(opt), dim)
    if need == 0:
        _lib.check(L.uot_sinkhorn_implicit_backward(ctypes.byref(prob), ctypes.byref(opt), None, None, None, None,
                                                    None, None, 0, None, None, dim, None, None, None, 0, None))
    ws = _workspace(need, device)
    out = Gradients()
    out.grad_a = torch.empty(n, dtype=torch.float64, device=device) if want_a else None
    out.grad_b = torch.empty(m, dtype=torch.float64, device=device) if want_b else None
    out.grad_x = torch.empty((n, dim), dtype=torch.float64, device=device) if (x is not None and want_x) else None
    out.grad_y = torch.empty((m, dim), dtype=torch.float64, device=device) if (x is not None and want_y) else None
    out.grad_C = torch.empty((n, m), dtype=torch.float64, device=device) if want_C else None
    _lib.check(L.uot_sinkhorn_implicit_backward(ctypes.byref(prob), ctypes.byref(opt), _ptr(res.u), _ptr(res.v),
                                                _ptr(g), _ptr(out.grad_a), _ptr(out.grad_b), _ptr(out.grad_C), m,
                                                _ptr(x), _ptr(y), dim, _ptr(out.grad_x), _ptr(out.grad_y),
                                                _ptr(ws), ws.numel(), _stream(device)))
    out._keep = (ws, g, x, y, res)
    return out


class UOTLoss(torch.autograd.Function):
    """UOT objective of the unrolled loop on points, with gradients w.r.t. the
    source points x, the target points y and the histograms a and b.

    Forward: squared-Euclidean cost of (x, y) (not normalised), Gibbs kernel
    in ``k_dtype``, ``max_iter`` fused iterations with v and K^T u saved every
    ``checkpoint_every`` (0: every iterate kept, so that the reverse pass
    repeats no forward pass); backward: the library's reverse pass (dL/dy
    through the dense cost gradient, formed only when y needs a gradient)."""

    @staticmethod
    def forward(ctx, x, y, a, b, eps: float, tau: float, max_iter: int, checkpoint_every: int = 50,
                k_dtype: torch.dtype = torch.float32, implicit: bool = False):
        x64 = x.detach().to(torch.float64).contiguous()
        y64 = y.detach().to(torch.float64).contiguous()
        C = cost_from_points(x64, y64, UOT_COST_SQEUCLID, False)
        K = kernel_from_cost(C, eps, k_dtype)
        del C
        store = not implicit and checkpoint_every == 0
        res = sinkhorn(a.detach().to(torch.float64).contiguous(), b.detach().to(torch.float64).contiguous(), K,
                       eps=eps, tau=tau, max_iter=max_iter, checkpoint_every=0 if implicit else checkpoint_every,
                       store_iterates=store)
        ctx.res = res
        ctx.implicit = implicit
        ctx.save_for_backward(x64, y64)
        ctx.dtypes = (x.dtype, y.dtype, a.dtype, b.dtype)
        return res.loss.clone().to(x.dtype)

    @staticmethod
    def backward(ctx, grad):
        x64, y64 = ctx.saved_tensors
        need_x, need_y, need_a, need_b = ctx.needs_input_grad[:4]
        pts = need_x or need_y
        fn = sinkhorn_implicit_backward if ctx.implicit else sinkhorn_backward
        gr = fn(ctx.res, grad.detach().to(torch.float64), x=x64 if pts else None, y=y64 if pts else None,
                want_a=need_a, want_b=need_b, want_x=need_x, want_y=need_y)
        xd, yd, ad, bd = ctx.dtypes
        cast = lambda t, d: t.to(d) if t is not None else None  # noqa: E731
        return (cast(gr.grad_x, xd), cast(gr.grad_y, yd), cast(gr.grad_a, ad), cast(gr.grad_b, bd),
                None, None, None, None, None, None)


class UOTCostLoss(torch.autograd.Function):
    """UOT objective of the unrolled loop on a dense FP64 cost C, with
    gradients w.r.t. C (dense, on the matrix cores), a and b
    (``checkpoint_every`` 0: every iterate kept, as for UOTLoss)."""

    @staticmethod
    def forward(ctx, C, a, b, eps: float, tau: float, max_iter: int, checkpoint_every: int = 50,
                k_dtype: torch.dtype = torch.float32):
        C64 = C.detach().to(torch.float64).contiguous()
        K = kernel_from_cost(C64, eps, k_dtype)
        res = sinkhorn(a.detach().to(torch.float64).contiguous(), b.detach().to(torch.float64).contiguous(), K,
                       m=C64.shape[1], eps=eps, tau=tau, max_iter=max_iter, checkpoint_every=checkpoint_every,
                       store_iterates=checkpoint_every == 0)
        ctx.res = res
        ctx.dtypes = (C.dtype, a.dtype, b.dtype)
        return res.loss.clone().to(C.dtype)

    @staticmethod
    def backward(ctx, grad):
        need_C, need_a, need_b = ctx.needs_input_grad[:3]
        gr = sinkhorn_backward(ctx.res, grad.detach().to(torch.float64), want_a=need_a, want_b=need_b,
                               want_C=need_C)
        cd, ad, bd = ctx.dtypes
        cast = lambda t, d: t.to(d) if t is not None else None  # noqa: E731
        return (cast(gr.grad_C, cd), cast(gr.grad_a, ad), cast(gr.grad_b, bd), None, None, None, None, None)


def uot_loss(x, y, a, b, eps: float, tau: float, max_iter: int, checkpoint_every: int = 50,
             k_dtype: torch.dtype = torch.float32, implicit: bool = False) -> torch.Tensor:
    """Differentiable UOT objective of two point clouds (see UOTLoss);
    ``implicit`` uses the envelope gradient at the final scalings (exact at
    convergence, no checkpoints) instead of the unrolled reverse sweep."""
    return UOTLoss.apply(x, y, a, b, eps, tau, max_iter, checkpoint_every, k_dtype, implicit)


def uot_loss_cost(C, a, b, eps: float, tau: float, max_iter: int, checkpoint_every: int = 50,
                  k_dtype: torch.dtype = torch.float32) -> torch.Tensor:
    """Differentiable UOT objective of a dense cost matrix (see UOTCostLoss)."""
    return UOTCostLoss.apply(C, a, b, eps, tau, max_iter, checkpoint_every, k_dtype)


from .batched import BatchedResult, BatchedSolver, sinkhorn_batched  # noqa: E402
