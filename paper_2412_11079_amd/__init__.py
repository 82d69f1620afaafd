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

__all__ = ["sinkhorn", "cost_from_points", "kernel_from_cost", "SinkhornResult", "UOTError", "lib_path",
           "UOT_F64", "UOT_F32", "UOT_BF16", "UOT_FP8_E4M3", "UOT_COST_SQEUCLID", "UOT_COST_COSINE"]

_DTYPES = {torch.float64: UOT_F64, torch.float32: UOT_F32}
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


@dataclass
class SinkhornResult:
    u: torch.Tensor
    v: torch.Tensor
    r: torch.Tensor
    c: torch.Tensor
    loss: torch.Tensor            # device FP64 scalar
    info_raw: torch.Tensor        # device bytes of uot_info
    profile: Optional[dict] = None

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
             profile: bool = False) -> SinkhornResult:
    """UOT Sinkhorn scaling loop on the GPU (see include/uot.h, uot_sinkhorn).

    ``K`` is an (n, ldk) FP32/FP64 kernel (as returned by kernel_from_cost);
    ``m`` is the logical column count (default ``b.shape[0]``).  Without K, the
    FP64 cost ``C`` is turned into a kernel of ``k_dtype`` inside the call."""
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
    opt.absorb_log_threshold = 0.0
    opt.checkpoint_every = 0
    opt.tune = int(tune)
    opt.u0 = None if u0 is None else _vec64(u0, "u0", n, device).data_ptr()
    opt.v0 = None if v0 is None else _vec64(v0, "v0", m, device).data_ptr()
    opt.persistent = 1 if persistent else 0
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
    out = _lib.Outputs(u.data_ptr(), v.data_ptr(), r.data_ptr(), c.data_ptr(), loss.data_ptr(), info.data_ptr())
    prof = None
    if profile:
        p = _lib.Profile()
        _lib.check(L.uot_sinkhorn_profiled(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(out), _ptr(ws),
                                           ws.numel(), _stream(device), ctypes.byref(p)))
        prof = {f: getattr(p, f) for f, _ in _lib.Profile._fields_}
    else:
        _lib.check(L.uot_sinkhorn(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(out), _ptr(ws), ws.numel(),
                                  _stream(device)))
    res = SinkhornResult(u=u, v=v, r=r, c=c, loss=loss, info_raw=info, profile=prof)
    res._keepalive = (ws, K, C, a, b)  # buffers must outlive the enqueued work
    return res
