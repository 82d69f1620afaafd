"""Reverse pass of the unrolled loop on the GPU against the FP64 oracle's
adjoint (same iteration count, same checkpoint-free definition).

Gradient errors are normwise, ||g - g_ref||_2 / ||g_ref||_2 (componentwise
is ill-posed near zero): <= 1e-9 with FP64 K, <= 1e-5 with FP32 K (the
stated gradient bar)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


def _norm_err(g, ref):
    g = np.asarray(g, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


def _oracle_grads(prob, T):
    C = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    K = oracle.kernel(C, prob.eps)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T, trace=True)
    ga, gb, G = oracle.adjoint(K, prob.a, prob.b, prob.eps, prob.tau, res)
    gx = oracle.grad_points_sqeuclid(G, prob.x, prob.y)
    return res, ga, gb, gx


def _gpu_grads(prob, T, k, k_dtype, with_x=True):
    x, y = to_dev(prob.x), to_dev(prob.y)
    C = uot.cost_from_points(x, y, prob.cost_kind, prob.normalize_max)
    K = uot.kernel_from_cost(C, prob.eps, k_dtype)
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=T,
                       checkpoint_every=k)
    g = torch.ones((), dtype=torch.float64, device="cuda")
    ga, gb, gx = uot.sinkhorn_backward(res, g, x=x if with_x else None, y=y if with_x else None)
    torch.cuda.synchronize()
    return res, ga.cpu().numpy(), gb.cpu().numpy(), (gx.cpu().numpy() if gx is not None else None)


@pytest.mark.parametrize("n,m,T,k", [(300, 257, 20, 7), (129, 700, 9, 9), (64, 64, 1, 1)])
def test_backward_fp64_matches_oracle_adjoint(n, m, T, k):
    prob = workloads.grad(n=n, m=m, max_iter=T)
    say(f"backward FP64 n={n} m={m} T={T} k={k}")
    ref, ga0, gb0, gx0 = _oracle_grads(prob, T)
    res, ga, gb, gx = _gpu_grads(prob, T, k, torch.float64)
    assert abs(float(res.loss.cpu()) - ref.loss) <= 1e-12 * abs(ref.loss)
    for name, g, r in (("a", ga, ga0), ("b", gb, gb0), ("x", gx, gx0)):
        e = _norm_err(g, r)
        say(f"  grad_{name}: {e:.3e}")
        assert e <= 1e-9, name


@pytest.mark.parametrize("n,m,T,k", [(1000, 1500, 40, 8), (777, 4093, 25, 10)])
def test_backward_fp32_matches_oracle_adjoint(n, m, T, k):
    prob = workloads.grad(n=n, m=m, max_iter=T)
    say(f"backward FP32 n={n} m={m} T={T} k={k}")
    ref, ga0, gb0, gx0 = _oracle_grads(prob, T)
    res, ga, gb, gx = _gpu_grads(prob, T, k, torch.float32)
    for name, g, r in (("a", ga, ga0), ("b", gb, gb0), ("x", gx, gx0)):
        e = _norm_err(g, r)
        say(f"  grad_{name}: {e:.3e}")
        assert e <= 1e-5, name


def test_backward_two_dimensional_points_and_no_points():
    prob = workloads.plain_fp64(n=200, m=333)
    prob.max_iter = 15
    ref, ga0, gb0, gx0 = _oracle_grads(prob, 15)
    res, ga, gb, gx = _gpu_grads(prob, 15, 4, torch.float64)
    assert _norm_err(gx, gx0) <= 1e-9 and _norm_err(ga, ga0) <= 1e-9 and _norm_err(gb, gb0) <= 1e-9
    res2, ga2, gb2, gx2 = _gpu_grads(prob, 15, 4, torch.float64, with_x=False)
    assert gx2 is None
    assert _norm_err(ga2, ga0) <= 1e-9 and _norm_err(gb2, gb0) <= 1e-9


def test_checkpoint_interval_does_not_change_gradients():
    prob = workloads.grad(n=500, m=640, max_iter=24)
    outs = [_gpu_grads(prob, 24, k, torch.float32)[1:] for k in (1, 5, 24)]
    for o in outs[1:]:
        for g, g0 in zip(o, outs[0]):
            assert np.array_equal(g, g0)


def test_autograd_function_matches_direct_call():
    prob = workloads.grad(n=400, m=300, max_iter=30)
    x = to_dev(prob.x).requires_grad_(True)
    y = to_dev(prob.y)
    a = to_dev(prob.a).requires_grad_(True)
    b = to_dev(prob.b).requires_grad_(True)
    L = uot.uot_loss(x, y, a, b, prob.eps, prob.tau, 30, checkpoint_every=10, k_dtype=torch.float64)
    (2.5 * L).backward()
    _, ga, gb, gx = _gpu_grads(prob, 30, 10, torch.float64)
    np.testing.assert_allclose(x.grad.cpu().numpy(), 2.5 * gx, rtol=1e-14, atol=0)
    np.testing.assert_allclose(a.grad.cpu().numpy(), 2.5 * ga, rtol=1e-14, atol=0)
    np.testing.assert_allclose(b.grad.cpu().numpy(), 2.5 * gb, rtol=1e-14, atol=0)


def test_backward_argument_errors():
    prob = workloads.grad(n=64, m=64, max_iter=5)
    x, y = to_dev(prob.x), to_dev(prob.y)
    C = uot.cost_from_points(x, y)
    K = uot.kernel_from_cost(C, prob.eps, torch.float32)
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, eps=prob.eps, tau=prob.tau, max_iter=5)
    g = torch.ones((), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        uot.sinkhorn_backward(res, g)            # no checkpoints in the forward
    with pytest.raises(uot.UOTError):
        uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, eps=prob.eps, tau=prob.tau, max_iter=5,
                     checkpoint_every=2, tol=1e-6)


def test_backward_directional_finite_differences_gpu():
    """Self-consistency: the GPU gradient against central differences of the
    GPU forward (FP64 K, h = 1e-4 relative steps), along random directions."""
    prob = workloads.grad(n=1024, m=1024, max_iter=60)
    x, y = to_dev(prob.x), to_dev(prob.y)
    a, b = to_dev(prob.a), to_dev(prob.b)
    res, ga, gb, gx = _gpu_grads(prob, 60, 10, torch.float64)

    def loss(xx, aa, bb):
        C = uot.cost_from_points(xx, y)
        K = uot.kernel_from_cost(C, prob.eps, torch.float64)
        r = uot.sinkhorn(aa, bb, K, eps=prob.eps, tau=prob.tau, max_iter=60)
        return float(r.loss.cpu())

    rng = np.random.default_rng(7)
    h = 1e-4
    for _ in range(3):
        dx = rng.standard_normal(prob.x.shape)
        dx /= np.linalg.norm(dx)
        fd = (loss(x + h * to_dev(dx), a, b) - loss(x - h * to_dev(dx), a, b)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(gx * dx)), rel=1e-6, abs=1e-10)
        da = rng.standard_normal(prob.n) * prob.a          # relative steps keep a > 0
        fd = (loss(x, a + h * to_dev(da), b) - loss(x, a - h * to_dev(da), b)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(ga * da)), rel=1e-6, abs=1e-12)
        db = rng.standard_normal(prob.m) * prob.b
        fd = (loss(x, a, b + h * to_dev(db)) - loss(x, a, b - h * to_dev(db))) / (2 * h)
        assert fd == pytest.approx(float(np.sum(gb * db)), rel=1e-6, abs=1e-12)


def test_backward_full_size_against_oracle():
    """Differentiation workload at full size: 8192^2 FP32, 500 iterations,
    checkpoints every 50, against the oracle's adjoint run at full size."""
    prob = workloads.grad()
    say("full-size backward: oracle adjoint on the host ...")
    ref, ga0, gb0, gx0 = _oracle_grads(prob, prob.max_iter)
    say("  GPU ...")
    res, ga, gb, gx = _gpu_grads(prob, prob.max_iter, prob.checkpoint_every, torch.float32)
    for name, g, r in (("a", ga, ga0), ("b", gb, gb0), ("x", gx, gx0)):
        e = _norm_err(g, r)
        say(f"  grad_{name}: {e:.3e}")
        assert e <= 1e-5, name
