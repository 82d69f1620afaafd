"""Log-domain solve (uot_sinkhorn_lse): potentials carried through
log-sum-exp passes over the stored cost, with an optional eps-scaling
schedule, against the FP64 log-domain oracle (orc_sinkhorn_lse, pinned to
the vector form, the 1x1 and rank-1 closed forms) on the same cost.

Errors are those of the totals u = e^{f/eps}, v = e^{g/eps}: entrywise
max |e^{(f - f_ref)/eps} - 1|.  Bars: every exponential is the hardware
exp2 on an FP32 argument taken under its row or column maximum, so each
term carries a relative error of about 2^-24 on the terms that matter,
like an FP32-stored kernel: 1e-6 where the fixed point does not amplify
(fi <= 0.95), and the stored kernel's own bound 2 fi/(1 - fi) 2^-24 at
the precision workload (fi = 0.990); the loss and marginals 1e-6.  An FP32
cost is compared with the oracle run on the same FP32-rounded cost.
Shapes cover 1, 2 and 4 chunks per lane (FP64) and 1 and 2 (FP32), ragged
row and column counts, a single row and column."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    say(f"libuot: {uot.lib_path()}")


def _pot_err(f, f0, eps):
    """Entrywise relative error of e^{f/eps} (zeros must match)."""
    f, f0 = np.asarray(f), np.asarray(f0)
    z = np.isneginf(f0)
    assert np.array_equal(np.isneginf(f), z), "zero-mass pattern differs"
    return float(np.max(np.abs(np.expm1((f[~z] - f0[~z]) / eps)))) if np.any(~z) else 0.0


def _rel(x, x0):
    x, x0 = np.asarray(x), np.asarray(x0)
    nz = x0 != 0
    assert np.all(x[~nz] == 0)
    return float(np.max(np.abs(x[nz] / x0[nz] - 1))) if np.any(nz) else 0.0


def _compare(res, ref, eps, bar, what):
    eu = _pot_err(res.f.cpu().numpy(), ref.f, eps)
    ev = _pot_err(res.g.cpu().numpy(), ref.g, eps)
    el = abs(float(res.loss.cpu()) / ref.loss - 1)
    er = _rel(res.r.cpu().numpy(), ref.r)
    ec = _rel(res.c.cpu().numpy(), ref.c)
    say(f"  {what}: u {eu:.3e} v {ev:.3e} loss {el:.3e} r {er:.3e} c {ec:.3e}")
    assert eu <= bar and ev <= bar, what
    assert el <= 1e-6 and er <= max(bar, 1e-6) and ec <= max(bar, 1e-6), what


def _solve(C, a, b, eps, tau, T, cost_dtype=torch.float64, **kw):
    r = uot.sinkhorn_lse(to_dev(C), to_dev(a), to_dev(b), eps=eps, tau=tau, max_iter=T, cost_dtype=cost_dtype, **kw)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("n,m,cost_dtype", [(1000, 777, torch.float64), (257, 2048, torch.float64),
                                            (300, 2049, torch.float64), (3001, 4097, torch.float64),
                                            (100, 8192, torch.float64), (1, 1, torch.float64),
                                            (2, 3, torch.float64), (999, 1000, torch.float32),
                                            (500, 4096, torch.float32), (777, 4097, torch.float32),
                                            (64, 8192, torch.float32)])
def test_shapes_against_oracle(n, m, cost_dtype):
    prob = workloads.random_small(n, m, seed=8000 + n + m, eps=0.02, tau=1.0, d=3)
    C = oracle.cost_points(prob.x, prob.y)
    if cost_dtype == torch.float32:
        C = C.astype(np.float32).astype(np.float64)     # the cost the passes read
    say(f"lse n={n} m={m} {cost_dtype}")
    ref = oracle.sinkhorn_lse(C, prob.a, prob.b, prob.eps, prob.tau, 30)
    res = _solve(C, prob.a, prob.b, prob.eps, prob.tau, 30, cost_dtype)
    info = res.info()
    assert info["iters"] == 30 and info["flags"] == 0, info
    _compare(res, ref, prob.eps, 1e-6, f"{n}x{m}")
    # the totals: e^{f/eps}
    u = res.u.cpu().numpy()
    assert _rel(u, np.exp(ref.f / prob.eps)) <= 1e-6


def test_small_eps_where_the_kernel_underflows():
    """eps = 1e-3 on costs in [0, 3): kernel entries down to e^-3000 (FP64
    underflow for the vector form); unbalanced and balanced."""
    for tau in (1.0, math.inf):
        prob = workloads.random_small(1500, 3000, seed=8101, eps=1e-3, tau=tau, d=3)
        C = oracle.cost_points(prob.x, prob.y)
        ref = oracle.sinkhorn_lse(C, prob.a, prob.b, 1e-3, tau, 40)
        res = _solve(C, prob.a, prob.b, 1e-3, tau, 40)
        assert res.info()["flags"] == 0
        fi = oracle.fi_exponent(1e-3, tau)
        bar = 1e-6 if fi < 0.99 else 2e-5
        _compare(res, ref, 1e-3, bar if not math.isinf(tau) else 5e-5, f"eps 1e-3 tau={tau}")


def test_zero_mass_entries():
    prob = workloads.random_small(600, 700, seed=8102, eps=0.05, tau=1.0, d=2)
    a, b = prob.a.copy(), prob.b.copy()
    a[::5] = 0.0
    b[::7] = 0.0
    C = oracle.cost_points(prob.x, prob.y)
    ref = oracle.sinkhorn_lse(C, a, b, prob.eps, prob.tau, 25)
    res = _solve(C, a, b, prob.eps, prob.tau, 25)
    assert np.all(res.u.cpu().numpy()[::5] == 0) and np.all(res.v.cpu().numpy()[::7] == 0)
    _compare(res, ref, prob.eps, 1e-6, "zero mass")


def test_tolerance_stop_matches_oracle_iteration():
    prob = workloads.random_small(900, 1100, seed=8103, eps=0.05, tau=1.0, d=2)
    C = oracle.cost_points(prob.x, prob.y)
    ref = oracle.sinkhorn_lse(C, prob.a, prob.b, prob.eps, prob.tau, 3000, tol=1e-6)
    assert 10 < ref.iters < 3000
    for every in (1, 3):
        res = _solve(C, prob.a, prob.b, prob.eps, prob.tau, 3000, tol=1e-6, check_every=every)
        info = res.info()
        say(f"  check_every={every}: GPU {info['iters']} oracle {ref.iters}")
        assert info["iters"] == ref.iters and info["err"] <= 1e-6 and info["flags"] == 0
        _compare(res, ref, prob.eps, 1e-6, "tol stop")
    res = _solve(C, prob.a, prob.b, prob.eps, prob.tau, 4, tol=1e-12)
    assert res.info()["flags"] & uot.UOT_FLAG_NOT_CONVERGED


def test_eps_scaling_schedule_against_oracle():
    """Stages 0.64, 0.32, ..., 0.01 (10 iterations each) then 40 at 0.005,
    and the tolerance stop at the last stage."""
    prob = workloads.random_small(1200, 900, seed=8104, eps=0.005, tau=0.5, d=3)
    C = oracle.cost_points(prob.x, prob.y)
    sch = dict(eps0=0.64, factor=0.5, stage_iters=10)
    ref = oracle.sinkhorn_lse(C, prob.a, prob.b, 0.005, 0.5, 40, **sch)
    res = _solve(C, prob.a, prob.b, 0.005, 0.5, 40, **sch)
    assert ref.iters == 7 * 10 + 40 and res.info()["iters"] == ref.iters
    _compare(res, ref, 0.005, 1e-6, "eps-scaling")
    ref = oracle.sinkhorn_lse(C, prob.a, prob.b, 0.005, 0.5, 5000, tol=1e-7, **sch)
    res = _solve(C, prob.a, prob.b, 0.005, 0.5, 5000, tol=1e-7, **sch)
    say(f"  scaled tol stop: GPU {res.info()['iters']} oracle {ref.iters}")
    assert res.info()["iters"] == ref.iters
    _compare(res, ref, 0.005, 1e-6, "eps-scaling tol")


def test_bitwise_reproducible():
    prob = workloads.random_small(3000, 5000, seed=8105, eps=0.01, tau=1.0, d=3)
    C = to_dev(oracle.cost_points(prob.x, prob.y))
    a, b = to_dev(prob.a), to_dev(prob.b)
    r1 = uot.sinkhorn_lse(C, a, b, eps=0.01, tau=1.0, max_iter=12)
    r2 = uot.sinkhorn_lse(C, a, b, eps=0.01, tau=1.0, max_iter=12)
    torch.cuda.synchronize()
    assert torch.equal(r1.f, r2.f) and torch.equal(r1.g, r2.g) and torch.equal(r1.loss, r2.loss)


def test_argument_errors():
    prob = workloads.random_small(10, 20, seed=8106, d=2)
    C = to_dev(oracle.cost_points(prob.x, prob.y))
    a, b = to_dev(prob.a), to_dev(prob.b)
    with pytest.raises(uot.UOTError, match="8192"):
        uot.sinkhorn_lse(torch.zeros((10, 8194), dtype=torch.float64, device=C.device), a,
                         to_dev(np.ones(8193)), m=8193, eps=0.1, tau=1.0, max_iter=1)
    with pytest.raises(uot.UOTError, match="factor"):
        uot.sinkhorn_lse(C, a, b, eps=0.1, tau=1.0, max_iter=1, eps0=1.0, factor=1.5, stage_iters=2)
    with pytest.raises(uot.UOTError, match="stage_iters"):
        uot.sinkhorn_lse(C, a, b, eps=0.1, tau=1.0, max_iter=1, eps0=1.0, factor=0.5, stage_iters=0)
    with pytest.raises(uot.UOTError, match="FP64 or FP32"):
        uot.sinkhorn_lse(C, a, b, eps=0.1, tau=1.0, max_iter=1, cost_dtype=torch.bfloat16)


def test_precision_workload_full_size():
    """65536 x 8192, 16-D points, eps 1e-3, tau 0.1, 2000 iterations, FP64
    cost, against the FP64 oracle's result at full size (tests/golden):
    the stored-kernel bar 2 fi/(1 - fi) 2^-24 entrywise on u and v, 1e-6 on
    the loss, with no absorption at all."""
    z = np.load(__file__.replace("test_gpu_lse.py", "golden/precision_65536x8192_fp64.npz"))
    prob = workloads.precision()
    assert int(z["n"]) == prob.n and int(z["m"]) == prob.m and int(z["iters"]) == prob.max_iter
    C = uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), prob.cost_kind, prob.normalize_max)
    say("  precision workload, FP64 cost, 2000 iterations ...")
    res = uot.sinkhorn_lse(C, to_dev(prob.a), to_dev(prob.b), eps=prob.eps, tau=prob.tau, max_iter=prob.max_iter)
    torch.cuda.synchronize()
    info = res.info()
    assert info["flags"] == 0 and info["iters"] == 2000
    eu = _pot_err(res.f.cpu().numpy(), z["f"], prob.eps)
    ev = _pot_err(res.g.cpu().numpy(), z["g"], prob.eps)
    el = abs(float(res.loss.cpu()) / float(z["loss"]) - 1)
    fi = prob.tau / (prob.tau + prob.eps)
    say(f"    vs FP64 oracle: u {eu:.3e} v {ev:.3e} loss {el:.3e}")
    assert max(eu, ev) <= 2 * fi / (1 - fi) * 2.0 ** -24 and el <= 1e-6
