"""Shared helpers of the GPU tests: run the HIP path on a workloads.Problem
and compare with the oracle.  Imported only by tests marked ``gpu``."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2412_11079_amd as uot

DEV = "cuda:0"


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def gpu_cost(prob) -> torch.Tensor:
    """FP64 cost on the GPU (library kernel for points; a separable cost is
    formed by the test with torch, it is input data, not solver work)."""
    if prob.x is not None:
        return uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), prob.cost_kind, prob.normalize_max)
    return (to_dev(prob.alpha)[:, None] + to_dev(prob.beta)[None, :]).contiguous()


def gpu_solve(prob, k_dtype=torch.float32, max_iter=None, tol=None, fused=True, check_every=1, tune=0,
              accum="f32", C=None, K=None, persistent=False):
    if C is None and K is None:
        C = gpu_cost(prob)
    if K is None:
        K = uot.kernel_from_cost(C, prob.eps, k_dtype)
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, m=prob.m, eps=prob.eps, tau=prob.tau,
                       max_iter=prob.max_iter if max_iter is None else max_iter,
                       tol=prob.tol if tol is None else tol, fused=fused, check_every=check_every,
                       tune=tune, accum=accum, persistent=persistent)
    torch.cuda.synchronize()
    return res, K


def rel_err(x: np.ndarray, ref: np.ndarray) -> float:
    """max_i |x_i / ref_i - 1| over entries with ref_i != 0 (zeros must match exactly)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    zero = ref == 0
    if np.any(x[zero] != 0):
        return float("inf")
    nz = ~zero
    if not np.any(nz):
        return 0.0
    return float(np.max(np.abs(x[nz] / ref[nz] - 1.0)))


def compare(res, ref, tol_uv: float, tol_loss: float, what: str = ""):
    u = res.u.cpu().numpy()
    v = res.v.cpu().numpy()
    L = float(res.loss.cpu())
    eu = rel_err(u, ref.u)
    ev = rel_err(v, ref.v)
    el = abs(L - ref.loss) / abs(ref.loss)
    say(f"  {what}: err u {eu:.3e}  v {ev:.3e}  loss {el:.3e}")
    assert eu <= tol_uv, f"{what}: u error {eu:.3e} > {tol_uv}"
    assert ev <= tol_uv, f"{what}: v error {ev:.3e} > {tol_uv}"
    assert el <= tol_loss, f"{what}: loss error {el:.3e} > {tol_loss}"
    return eu, ev, el
