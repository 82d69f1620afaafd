"""The no-allocation entry point (uot_sinkhorn_noalloc) against uot_sinkhorn,
called through the C-ABI with the same problem, options and kernel.

Both run the same kernels, so results must agree bit for bit: two calls in a
row (the second on a smaller problem, so stale scratch contents from the
first would show), a tolerance stop (launches after the stop return at once
instead of the host breaking the loop), and the size and absorption limits."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2412_11079_amd as uot
import workloads
from paper_2412_11079_amd import _lib
from gpu_helpers import DEV, gpu_cost, say, to_dev

pytestmark = pytest.mark.gpu


def _call(prob, K, max_iter, tol, noalloc, check_every=1, accum=_lib.UOT_ACC_F32):
    """One solve through the C-ABI; returns (u, v, r, c, loss, info dict)."""
    L = _lib.lib()
    a, b = to_dev(prob.a), to_dev(prob.b)
    p = _lib.Problem()
    p.n, p.m = prob.n, prob.m
    p.a, p.b = a.data_ptr(), b.data_ptr()
    p.k_dtype = _lib.UOT_F32
    p.K = K.data_ptr()
    p.ldk = K.stride(0)
    p.eps, p.tau, p.k_scale = prob.eps, prob.tau, 1.0
    o = _lib.Options()
    o.max_iter, o.check_every, o.tol, o.fused, o.accum = max_iter, check_every, tol, 1, accum
    outs = {k: torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
            for k, n in (("u", prob.n), ("v", prob.m), ("r", prob.n), ("c", prob.m))}
    loss = torch.full((), float("nan"), dtype=torch.float64, device=DEV)
    info = torch.zeros(ctypes.sizeof(_lib.Info), dtype=torch.uint8, device=DEV)
    out = _lib.Outputs(outs["u"].data_ptr(), outs["v"].data_ptr(), outs["r"].data_ptr(), outs["c"].data_ptr(),
                       loss.data_ptr(), info.data_ptr(), None, None, None)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        st = L.uot_sinkhorn_noalloc(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out), stream)
    else:
        need = L.uot_sinkhorn_workspace_size(ctypes.byref(p), ctypes.byref(o))
        ws = torch.empty(need, dtype=torch.uint8, device=DEV)
        st = L.uot_sinkhorn(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()),
                            need, stream)
    _lib.check(st)
    torch.cuda.synchronize()
    inf = _lib.Info.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))
    res = {k: t.cpu().numpy() for k, t in outs.items()}
    res["loss"] = float(loss.cpu())
    res["info"] = (int(inf.iters), float(inf.err), int(inf.flags))
    return res


def _kernel(prob):
    return uot.kernel_from_cost(gpu_cost(prob), prob.eps, torch.float32)


def _same(x, y, what):
    for k in ("u", "v", "r", "c"):
        assert np.array_equal(x[k], y[k]), f"{what}: {k} differs (max {np.max(np.abs(x[k] - y[k])):.3e})"
    assert x["loss"] == y["loss"], f"{what}: loss {x['loss']!r} vs {y['loss']!r}"
    assert x["info"] == y["info"], f"{what}: info {x['info']} vs {y['info']}"


def test_noalloc_matches_workspace_call_twice_in_a_row():
    big = workloads.headline(n=4096, m=5000, max_iter=60)
    small = workloads.headline(n=777, m=1531, max_iter=25)
    Kb, Ks = _kernel(big), _kernel(small)
    torch.cuda.synchronize()
    for prob, K, what in ((big, Kb, "4096 x 5000"), (small, Ks, "777 x 1531")):
        say(f"no-alloc vs workspace call, {what}, {prob.max_iter} iterations")
        ref = _call(prob, K, prob.max_iter, 0.0, noalloc=False)
        got = _call(prob, K, prob.max_iter, 0.0, noalloc=True)
        assert np.all(np.isfinite(got["u"])) and np.all(np.isfinite(got["v"]))
        _same(got, ref, what)


def test_noalloc_tolerance_stop_matches():
    prob = workloads.headline(n=1500, m=2100, max_iter=400)
    K = _kernel(prob)
    say("no-alloc tolerance stop, 1500 x 2100, tol 1e-6, check every 3")
    ref = _call(prob, K, 400, 1e-6, noalloc=False, check_every=3)
    got = _call(prob, K, 400, 1e-6, noalloc=True, check_every=3)
    assert 1 < ref["info"][0] < 400, ref["info"]
    _same(got, ref, "tol stop")


def test_noalloc_fp64_accumulation_and_limits():
    prob = workloads.headline(n=600, m=900, max_iter=30)
    K = _kernel(prob)
    ref = _call(prob, K, 30, 0.0, noalloc=False, accum=_lib.UOT_ACC_F64)
    got = _call(prob, K, 30, 0.0, noalloc=True, accum=_lib.UOT_ACC_F64)
    _same(got, ref, "FP64 accumulation")
    # A problem whose workspace exceeds the scratch is refused before any launch:
    # a kernel built inside the call from C (4096 x 16384 FP32, 256 MiB).
    L = _lib.lib()
    p = _lib.Problem()
    p.n, p.m = 4096, 16384
    a = torch.ones(p.n, dtype=torch.float64, device=DEV)
    b = torch.ones(p.m, dtype=torch.float64, device=DEV)
    p.a, p.b = a.data_ptr(), b.data_ptr()
    p.k_dtype, p.K, p.ldk = _lib.UOT_F32, None, 0
    p.C, p.ldc = a.data_ptr(), p.m          # never read: the call is refused first
    p.eps, p.tau = 0.01, 0.5
    o = _lib.Options()
    o.max_iter, o.check_every, o.fused = 1, 1, 1
    need = L.uot_sinkhorn_workspace_size(ctypes.byref(p), ctypes.byref(o))
    assert need > _lib.UOT_NOALLOC_SCRATCH_BYTES, need
    u = torch.empty(p.n, dtype=torch.float64, device=DEV)
    v = torch.empty(p.m, dtype=torch.float64, device=DEV)
    out = _lib.Outputs(u.data_ptr(), v.data_ptr(), None, None, None, None, None, None, None)
    st = L.uot_sinkhorn_noalloc(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out), None)
    assert st == _lib.UOT_ERR_WORKSPACE, st
    assert b"scratch" in L.uot_last_error()
    # absorption decides on the host: refused
    o.absorb_log_threshold = 30.0
    st = L.uot_sinkhorn_noalloc(ctypes.byref(p), ctypes.byref(o), ctypes.byref(out), None)
    assert st == _lib.UOT_ERR_UNSUPPORTED, st
