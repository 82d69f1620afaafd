"""Dense plan output P = diag(u) K diag(v) against the oracle's plan, and its
margins against the solve's marginals."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import gpu_solve, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


def _oracle_plan(prob):
    res, C, K = oracle.solve_problem(prob)
    return res, C, res.u[:, None] * K * res.v[None, :]


@pytest.mark.parametrize("k_dtype,plan_dtype,bar", [(torch.float64, torch.float64, 1e-12),
                                                    (torch.float64, torch.float32, 2 ** -24 * 1.01 + 1e-12),
                                                    (torch.float32, torch.float64, 3e-6)])
def test_plan_from_kernel_matches_oracle(k_dtype, plan_dtype, bar):
    prob = workloads.plain_fp64(n=300, m=257)
    ref, C, P0 = _oracle_plan(prob)
    res, K = gpu_solve(prob, k_dtype=k_dtype)
    P = uot.plan(res, dtype=plan_dtype).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    big = P0 > 1e-300
    e = float(np.max(np.abs(P[big] / P0[big] - 1)))
    say(f"  K {k_dtype}, plan {plan_dtype}: {e:.3e}")
    assert e <= bar
    if plan_dtype == torch.float64:
        # the solve's marginals come from its own passes: FP32 lane sums with an FP32 K
        rt = 1e-12 if k_dtype == torch.float64 else 1e-6
        np.testing.assert_allclose(P.sum(axis=1), res.r.cpu().numpy(), rtol=rt)
        np.testing.assert_allclose(P.sum(axis=0), res.c.cpu().numpy(), rtol=rt)


def test_plan_from_cost_after_absorption():
    prob = workloads.precision(n=1024, m=512, max_iter=120)
    ref, C, _ = oracle.solve_problem(prob)
    f0, g0 = prob.eps * np.log(ref.u), prob.eps * np.log(ref.v)
    P0 = np.exp((f0[:, None] + g0[None, :] - C) / prob.eps)
    Cd = uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), prob.cost_kind, prob.normalize_max)
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), None, C=Cd, k_dtype=torch.float64, eps=prob.eps,
                       tau=prob.tau, max_iter=prob.max_iter, absorb_log_threshold=30.0)
    P = uot.plan(res, from_cost=True).cpu().numpy()
    torch.cuda.synchronize()
    assert res.info()["absorptions"] >= 1
    sig = P0 > 1e-12 * P0.max()
    e = float(np.max(np.abs(P[sig] / P0[sig] - 1)))
    say(f"  plan from potentials: {e:.3e}")
    assert e <= 1e-10
    np.testing.assert_allclose(P.sum(axis=1), res.r.cpu().numpy(), rtol=1e-10)
    np.testing.assert_allclose(P.sum(axis=0), res.c.cpu().numpy(), rtol=1e-10)


def test_plan_argument_errors():
    prob = workloads.plain_fp64(n=64, m=64)
    res, K = gpu_solve(prob, k_dtype=torch.float32)
    with pytest.raises(ValueError):
        uot.plan(res, dtype=torch.bfloat16)
    with pytest.raises(ValueError):
        uot.plan(res, from_cost=True)        # the solve had no C
