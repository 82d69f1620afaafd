"""Two solves at once from two host threads on two streams (same, default
priority): one stopping on a tolerance (the host reads a pinned flag every
few iterations), one with log-domain absorption (the host reads pinned
maxima at every check), with profiling on both.  Each call holds its own
pinned words and events, so the results equal the same solves run one
after the other, bit for bit."""
import threading

import pytest
import torch

import workloads
from gpu_helpers import gpu_cost, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


def _solve_tol(prob, K):
    return uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, m=prob.m, eps=prob.eps, tau=prob.tau,
                        max_iter=prob.max_iter, tol=prob.tol, check_every=3, profile=True)


def _solve_absorbed(prob, C):
    return uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), None, C=C, k_dtype=torch.bfloat16, eps=prob.eps,
                        tau=prob.tau, max_iter=prob.max_iter, absorb_log_threshold=30.0, check_every=5,
                        profile=True)


def _snap(res):
    torch.cuda.synchronize()
    return {"u": res.u.clone(), "v": res.v.clone(), "loss": float(res.loss), "info": res.info()}


def test_two_threads_two_streams_equal_serial_runs():
    p1 = workloads.headline(n=3000, m=4000, max_iter=600, tol=1e-6)
    p2 = workloads.precision(n=2048, m=1024, max_iter=200)
    K1 = uot.kernel_from_cost(gpu_cost(p1), p1.eps, torch.float32)
    C2 = gpu_cost(p2)
    torch.cuda.synchronize()
    say("serial runs ...")
    ref1 = _snap(_solve_tol(p1, K1))
    ref2 = _snap(_solve_absorbed(p2, C2))
    assert 1 < ref1["info"]["iters"] < 600 and ref2["info"]["absorptions"] >= 1

    out = {}
    errors = []

    def run(key, fn):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    r = fn()
                    s.synchronize()
                    out.setdefault(key, []).append({"u": r.u.clone(), "v": r.v.clone(), "loss": float(r.loss),
                                                    "info": r.info()})
                    s.synchronize()
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    say("two threads ...")
    t1 = threading.Thread(target=run, args=("tol", lambda: _solve_tol(p1, K1)))
    t2 = threading.Thread(target=run, args=("abs", lambda: _solve_absorbed(p2, C2)))
    t1.start()
    t2.start()
    t1.join(timeout=120)
    t2.join(timeout=120)
    assert not t1.is_alive() and not t2.is_alive()
    torch.cuda.synchronize()
    assert not errors, errors
    for key, ref in (("tol", ref1), ("abs", ref2)):
        assert len(out[key]) == 3
        for got in out[key]:
            assert torch.equal(got["u"], ref["u"]) and torch.equal(got["v"], ref["v"]), key
            assert got["loss"] == ref["loss"] and got["info"] == ref["info"], key


def test_kernel_free_and_log_domain_solves_in_two_threads():
    """The kernel-free solve and the log-domain solve, both stopping on a
    tolerance (pinned flag reads), from two host threads on two streams:
    equal to the serial runs bit for bit."""
    import oracle
    p1 = workloads.random_small(2000, 3000, seed=9101, eps=0.05, tau=1.0, d=3)
    p2 = workloads.random_small(1500, 1200, seed=9102, eps=0.01, tau=1.0, d=2)
    x1, y1, a1, b1 = to_dev(p1.x), to_dev(p1.y), to_dev(p1.a), to_dev(p1.b)
    C2, a2, b2 = to_dev(oracle.cost_points(p2.x, p2.y)), to_dev(p2.a), to_dev(p2.b)

    def kf():
        return uot.sinkhorn_points(x1, y1, a1, b1, eps=p1.eps, tau=p1.tau, max_iter=3000, tol=1e-6, check_every=3)

    def lse():
        return uot.sinkhorn_lse(C2, a2, b2, eps=p2.eps, tau=p2.tau, max_iter=3000, tol=1e-6, check_every=4,
                                eps0=0.2, factor=0.5, stage_iters=5)

    ref1 = _snap(kf())
    ref2 = _snap(lse())
    assert 1 < ref1["info"]["iters"] < 3000 and 1 < ref2["info"]["iters"] < 3000
    out, errors = {}, []

    def run(key, fn):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    r = fn()
                    s.synchronize()
                    out.setdefault(key, []).append({"u": r.u.clone(), "v": r.v.clone(), "loss": float(r.loss),
                                                    "info": r.info()})
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    t1 = threading.Thread(target=run, args=("kf", kf))
    t2 = threading.Thread(target=run, args=("lse", lse))
    t1.start()
    t2.start()
    t1.join(timeout=120)
    t2.join(timeout=120)
    assert not t1.is_alive() and not t2.is_alive()
    torch.cuda.synchronize()
    assert not errors, errors
    for key, ref in (("kf", ref1), ("lse", ref2)):
        assert len(out[key]) == 3
        for got in out[key]:
            assert torch.equal(got["u"], ref["u"]) and torch.equal(got["v"], ref["v"]), key
            assert got["loss"] == ref["loss"] and got["info"] == ref["info"], key
