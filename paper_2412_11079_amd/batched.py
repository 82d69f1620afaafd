"""Batched problems of uneven size in one persistent launch (include/uot.h,
uot_sinkhorn_batched and its packed form).  Argument marshalling only."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Union

import numpy as np
import torch

from . import _lib
from ._lib import UOT_FP8_E4M3


def _as_list(x, count, name):
    if isinstance(x, (int, float)):
        return [float(x)] * count
    x = list(x)
    if len(x) != count:
        raise ValueError(f"{name} must be a scalar or have one entry per problem")
    return [float(v) for v in x]


@dataclass
class BatchedResult:
    """Per-problem results, packed: problem i owns u[u_off[i]:u_off[i]+n_i]
    (likewise r) and v[v_off[i]:v_off[i]+m_i] (likewise c)."""
    u: torch.Tensor
    v: torch.Tensor
    r: torch.Tensor
    c: torch.Tensor
    loss: torch.Tensor          # (count,) FP64
    info_raw: torch.Tensor      # (count, sizeof(uot_info)) bytes
    u_off: List[int]
    v_off: List[int]
    ns: List[int]
    ms: List[int]

    def problem(self, i: int):
        n, m, uo, vo = self.ns[i], self.ms[i], self.u_off[i], self.v_off[i]
        return self.u[uo:uo + n], self.v[vo:vo + m], self.r[uo:uo + n], self.c[vo:vo + m]

    def info(self, i: int) -> dict:
        raw = bytes(self.info_raw[i].cpu().numpy().tobytes())
        s = _lib.Info.from_buffer_copy(raw)
        return {"iters": s.iters, "err": s.err, "absorptions": s.absorptions, "flags": s.flags}


class BatchedSolver:
    """Holds the descriptors, outputs and workspace of a batch so that
    ``run()`` (two kernel launches, no host synchronisation, no copies) can
    be replayed or captured in a ``torch.cuda.CUDAGraph``.

    ``Ks``: list of (n_i, ldk_i) device tensors of one dtype (e.g. from
    ``kernel_from_cost``; m_i = ``b_list[i].shape[0]`` columns are used),
    ``a_list`` / ``b_list``: FP64 device vectors."""

    def __init__(self, Ks: Sequence[torch.Tensor], a_list: Sequence[torch.Tensor], b_list: Sequence[torch.Tensor],
                 *, eps: Union[float, Sequence[float]], tau: Union[float, Sequence[float]], max_iter: int,
                 tol: float = 0.0, check_every: int = 1, tune: int = 0, trace: bool = False):
        count = len(Ks)
        if len(a_list) != count or len(b_list) != count:
            raise ValueError("Ks, a_list and b_list must have one entry per problem")
        if count == 0:
            raise ValueError("empty batch")
        device = Ks[0].device
        dtype = Ks[0].dtype
        from . import _DTYPES, FP8_STORE_SCALE, _stream, _workspace
        if dtype not in _DTYPES:
            raise ValueError(f"unsupported K dtype {dtype}")
        eps_l = _as_list(eps, count, "eps")
        tau_l = _as_list(tau, count, "tau")
        self.ns = [int(a.shape[0]) for a in a_list]
        self.ms = [int(b.shape[0]) for b in b_list]
        self.u_off = list(np.concatenate([[0], np.cumsum(self.ns)[:-1]]).astype(int))
        self.v_off = list(np.concatenate([[0], np.cumsum(self.ms)[:-1]]).astype(int))
        N, M = sum(self.ns), sum(self.ms)
        f64 = dict(dtype=torch.float64, device=device)
        self.u = torch.empty(N, **f64)
        self.v = torch.empty(M, **f64)
        self.r = torch.empty(N, **f64)
        self.c = torch.empty(M, **f64)
        self.loss = torch.empty(count, **f64)
        isz = ctypes.sizeof(_lib.Info)
        self.info_raw = torch.zeros((count, isz), dtype=torch.uint8, device=device)
        probs = (_lib.Problem * count)()
        outs = (_lib.Outputs * count)()
        for i in range(count):
            K, a, b = Ks[i], a_list[i], b_list[i]
            if K.dtype != dtype or K.device != device:
                raise ValueError("all K must share one dtype and device")
            if a.dtype != torch.float64 or b.dtype != torch.float64 or not a.is_contiguous() or not b.is_contiguous():
                raise ValueError("a and b must be contiguous float64 vectors")
            n, m = self.ns[i], self.ms[i]
            if K.dim() != 2 or K.shape[0] != n or K.shape[1] < m or K.stride(1) != 1:
                raise ValueError(f"K[{i}] must be an (n, ldk >= m) row-major matrix")
            p = probs[i]
            p.n, p.m = n, m
            p.a, p.b = a.data_ptr(), b.data_ptr()
            p.k_dtype = _DTYPES[dtype]
            p.K = K.data_ptr()
            p.ldk = K.stride(0)
            p.eps, p.tau = eps_l[i], tau_l[i]
            p.k_scale = 1.0 / FP8_STORE_SCALE if _DTYPES[dtype] == UOT_FP8_E4M3 else 1.0
            uo, vo = self.u_off[i], self.v_off[i]
            o = outs[i]
            o.u = self.u[uo:].data_ptr()
            o.v = self.v[vo:].data_ptr()
            o.r = self.r[uo:].data_ptr()
            o.c = self.c[vo:].data_ptr()
            o.loss = self.loss[i:].data_ptr()
            o.info = self.info_raw[i].data_ptr()
        opt = _lib.Options()
        opt.max_iter = int(max_iter)
        opt.tol = float(tol)
        opt.check_every = int(check_every)
        opt.tune = int(tune)
        opt.fused = 1
        self.opt = opt
        L = _lib.lib()
        self.ws = _workspace(L.uot_sinkhorn_batched_workspace_size(count), device)
        if tune > 0:
            _lib.check(L.uot_batched_tune(probs, count, ctypes.byref(opt), outs, ctypes.c_void_p(self.ws.data_ptr()),
                                          self.ws.numel(), _stream(device)))
        nbytes = L.uot_batched_desc_bytes(count)
        host = (ctypes.c_uint8 * nbytes)()
        _lib.check(L.uot_batched_pack(probs, count, ctypes.byref(opt), outs, host, nbytes))
        meta_off = nbytes - ctypes.sizeof(_lib.BatchedMeta)
        self.meta = _lib.BatchedMeta.from_buffer_copy(bytes(host)[meta_off:])
        self.desc = torch.frombuffer(bytearray(bytes(host)[:meta_off]), dtype=torch.uint8).to(device)
        items = int(self.meta.items)
        words = np.frombuffer(bytes(host)[:items * _DESC_WORDS * 8], dtype=np.int64).reshape(items, _DESC_WORDS)
        self.order = [int(x) for x in words[:, _DESC_INDEX_WORD]]      # problem of each queue entry
        self.trace = torch.zeros(2 * items, dtype=torch.int64, device=device) if trace else None
        self.count = count
        self.items = items
        self.nsplit = int(self.meta.nsplit)
        self.device = device
        self._keep = (list(Ks), list(a_list), list(b_list))

    def run(self) -> None:
        """Enqueue the queue reset and the persistent launch on the current stream."""
        from . import _stream
        L = _lib.lib()
        _lib.check(L.uot_sinkhorn_batched_packed(ctypes.c_void_p(self.desc.data_ptr()), ctypes.byref(self.meta),
                                                 ctypes.byref(self.opt), ctypes.c_void_p(self.ws.data_ptr()),
                                                 self.ws.numel(),
                                                 None if self.trace is None else ctypes.c_void_p(self.trace.data_ptr()),
                                                 _stream(self.device)))

    def result(self) -> BatchedResult:
        return BatchedResult(self.u, self.v, self.r, self.c, self.loss, self.info_raw, self.u_off, self.v_off,
                             self.ns, self.ms)

    def shapes(self) -> List[int]:
        """Tile shape assigned to each problem (caller's order)."""
        words = self.desc.cpu().numpy()[:self.items * _DESC_WORDS * 8].view(np.int64).reshape(self.items, _DESC_WORDS)
        shape_word = words[:, _DESC_SHAPE_WORD]
        out = [0] * self.count
        for q in range(self.items):
            out[self.order[q]] = int(shape_word[q] >> 32)
        return out

    def parts(self) -> List[int]:
        """Queue entries (workgroups) each problem runs on (caller's order)."""
        out = [0] * self.count
        for q in range(self.items):
            out[self.order[q]] += 1
        return out

    def tail_idle_fraction(self) -> Optional[float]:
        """1 - (sum of per-entry busy times) / (workgroups x makespan),
        from the device wall-clock stamps of the last traced run."""
        if self.trace is None:
            return None
        t = self.trace.cpu().numpy().reshape(-1, 2)
        busy = float(np.sum(t[:, 1] - t[:, 0]))
        span = float(t[:, 1].max() - t[:, 0].min())
        grid = min(self.items, _max_grid_estimate(self))
        return 1.0 - busy / (grid * span) if span > 0 else 0.0


# BatchDesc layout (csrc/batch.h, size and offsets asserted there): 22
# 8-byte words; word 16 packs fi_is_one (low half) and shape (high half),
# word 17 is the caller's index of the problem.
_DESC_WORDS = 22
_DESC_SHAPE_WORD = 16
_DESC_INDEX_WORD = 17


def _max_grid_estimate(solver: BatchedSolver) -> int:
    """Workgroups that ran: the busiest moment of the trace (stamps overlap)."""
    t = solver.trace.cpu().numpy().reshape(-1, 2)
    ev = sorted([(s, 1) for s in t[:, 0]] + [(e, -1) for e in t[:, 1]])
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return max(best, 1)


def sinkhorn_batched(Ks: Sequence[torch.Tensor], a_list: Sequence[torch.Tensor], b_list: Sequence[torch.Tensor],
                     *, eps: Union[float, Sequence[float]], tau: Union[float, Sequence[float]], max_iter: int,
                     tol: float = 0.0, check_every: int = 1, tune: int = 0) -> BatchedResult:
    """One call of uot_sinkhorn_batched (copies the descriptors and
    synchronises the stream once before the launch)."""
    count = len(Ks)
    from . import _DTYPES, FP8_STORE_SCALE, _stream, _workspace
    device = Ks[0].device
    dtype = Ks[0].dtype
    eps_l = _as_list(eps, count, "eps")
    tau_l = _as_list(tau, count, "tau")
    ns = [int(a.shape[0]) for a in a_list]
    ms = [int(b.shape[0]) for b in b_list]
    u_off = list(np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(int))
    v_off = list(np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(int))
    f64 = dict(dtype=torch.float64, device=device)
    U, V = torch.empty(sum(ns), **f64), torch.empty(sum(ms), **f64)
    R, Cm = torch.empty(sum(ns), **f64), torch.empty(sum(ms), **f64)
    loss = torch.empty(count, **f64)
    info = torch.zeros((count, ctypes.sizeof(_lib.Info)), dtype=torch.uint8, device=device)
    probs = (_lib.Problem * count)()
    outs = (_lib.Outputs * count)()
    for i in range(count):
        K, a, b = Ks[i], a_list[i], b_list[i]
        p = probs[i]
        p.n, p.m = ns[i], ms[i]
        p.a, p.b = a.data_ptr(), b.data_ptr()
        p.k_dtype = _DTYPES[K.dtype]
        p.K = K.data_ptr()
        p.ldk = K.stride(0)
        p.eps, p.tau = eps_l[i], tau_l[i]
        p.k_scale = 1.0 / FP8_STORE_SCALE if K.dtype == torch.float8_e4m3fn else 1.0
        o = outs[i]
        o.u, o.v = U[u_off[i]:].data_ptr(), V[v_off[i]:].data_ptr()
        o.r, o.c = R[u_off[i]:].data_ptr(), Cm[v_off[i]:].data_ptr()
        o.loss = loss[i:].data_ptr()
        o.info = info[i].data_ptr()
    opt = _lib.Options()
    opt.max_iter, opt.tol, opt.check_every, opt.tune, opt.fused = int(max_iter), float(tol), int(check_every), \
        int(tune), 1
    L = _lib.lib()
    ws = _workspace(L.uot_sinkhorn_batched_workspace_size(count), device)
    _lib.check(L.uot_sinkhorn_batched(probs, count, ctypes.byref(opt), outs, ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel(), _stream(device)))
    res = BatchedResult(U, V, R, Cm, loss, info, u_off, v_off, ns, ms)
    res._keep = (ws, list(Ks), list(a_list), list(b_list))
    return res


def wall_clock_khz() -> int:
    return int(_lib.lib().uot_device_wall_clock_khz())
