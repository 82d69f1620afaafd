"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: FP64 K 1e-12 relative on u, v and the objective; FP32 K 1e-6
(the stated bar for FP32-stored K).  Errors are max_i |x_i/x_ref,i - 1|.
Sizes span several workgroups, strips and a ragged column tail; the
full-size cases run the launch configuration the benchmark times."""
import math

import numpy as np
import pytest
import torch

import oracle
import pins
import workloads
from gpu_helpers import compare, gpu_cost, gpu_solve, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    say(f"libuot: {uot.lib_path()}")


def _oracle(prob, max_iter=None, tol=None):
    res, C, K = oracle.solve_problem(prob, max_iter=max_iter, tol=tol)
    return res


# ------------------------------------------------------------------ building blocks
def test_cost_from_points_matches_oracle():
    for prob in (workloads.plain_fp64(n=300, m=211), workloads.headline(n=257, m=300),
                 workloads.batched(count=1, lo=40, hi=90)[0]):
        say(f"cost {prob.name} {prob.n}x{prob.m} kind={prob.cost_kind} norm={prob.normalize_max}")
        C = gpu_cost(prob).cpu().numpy()
        Cref = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
        np.testing.assert_allclose(C, Cref, rtol=1e-13, atol=1e-15)


def test_kernel_build_rounds_fp64_exponent():
    prob = workloads.plain_fp64(n=123, m=517)
    Cref = oracle.cost_points(prob.x, prob.y, 0, False)
    Kref = oracle.kernel(Cref, prob.eps)
    C = to_dev(Cref)
    K64 = uot.kernel_from_cost(C, prob.eps, torch.float64)
    K32 = uot.kernel_from_cost(C, prob.eps, torch.float32)
    k64 = K64.cpu().numpy()
    k32 = K32.cpu().numpy()
    assert k64.shape[1] % 64 == 0 and np.all(k64[:, 517:] == 0) and np.all(k32[:, 517:] == 0)
    np.testing.assert_allclose(k64[:, :517], Kref, rtol=4e-16, atol=0)
    # FP32: the FP64 value rounded to nearest; allow one FP32 ulp for
    # exponent results that land on a rounding boundary
    ulp = np.spacing(Kref.astype(np.float32))
    assert np.all(np.abs(k32[:, :517].astype(np.float64) - Kref) <= ulp)


# ------------------------------------------------------------------ small / ragged parity
@pytest.mark.parametrize("fused", [True, False])
def test_plain_fp64_workload_fp64_kernel(fused):
    prob = workloads.plain_fp64()
    say(f"plain_fp64 FP64 K fused={fused}")
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float64, fused=fused)
    assert res.info()["iters"] == 100
    compare(res, ref, 1e-12, 1e-12, "FP64 K")


@pytest.mark.parametrize("fused", [True, False])
def test_plain_fp64_workload_fp32_kernel(fused):
    prob = workloads.plain_fp64()
    say(f"plain_fp64 FP32 K fused={fused}")
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float32, fused=fused)
    compare(res, ref, 1e-6, 1e-6, "FP32 K")


RAGGED = [(1, 1), (5, 3), (64, 7), (300, 333), (1000, 1531), (777, 4097), (2049, 8191)]


@pytest.mark.parametrize("n,m", RAGGED)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ragged_sizes_fused_and_plain(n, m, dtype):
    if dtype == torch.float64 and m > 8192:
        pytest.skip("FP64 rows are limited to 8192 columns")
    if n * m < 64:
        # the headline recipe divides the cost by its maximum, so a tiny
        # problem has an entry exp(-1/0.01) = 3.7e-44, below FP32's normal
        # range; use the unnormalised 2-D recipe there
        prob = workloads.plain_fp64(n=n, m=m)
        prob.max_iter = 30
    else:
        prob = workloads.headline(n=n, m=m, max_iter=30)
    ref = _oracle(prob)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    for fused in (True, False):
        say(f"ragged n={n} m={m} {dtype} fused={fused}")
        res, _ = gpu_solve(prob, k_dtype=dtype, fused=fused)
        compare(res, ref, tol, tol, f"n={n} m={m} fused={fused}")


@pytest.mark.parametrize("shape", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15])
def test_every_launch_shape(shape):
    """Each instantiated launch shape (tune index) on a problem it covers;
    600 rows give workgroups a partial last batch in the row-batched shapes."""
    cover = {1: 1024, 2: 2048, 3: 4096, 4: 8192, 5: 8192, 6: 16384, 7: 16384, 8: 16384,
             9: 8192, 10: 4096, 11: 2048, 12: 1024, 13: 8192, 14: 4096, 15: 2048}[shape]
    n = 600
    prob = workloads.headline(n=n, m=cover - 3, max_iter=12)
    ref = _oracle(prob)
    for fused in (True, False):
        say(f"shape {shape} m={prob.m} fused={fused}")
        res, _ = gpu_solve(prob, k_dtype=torch.float32, fused=fused, tune=shape)
        compare(res, ref, 1e-6, 1e-6, f"shape {shape}")


def test_fp64_accumulation_variant():
    prob = workloads.headline(n=700, m=2500, max_iter=40)
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float32, accum="f64")
    compare(res, ref, 1e-6, 1e-6, "FP32 K, FP64 lanes")


# ------------------------------------------------------------------ stopping and degenerate cases
def test_tolerance_stop_matches_oracle_iteration():
    prob = workloads.headline(n=900, m=1100, max_iter=2000, tol=1e-6)
    ref = _oracle(prob)
    say(f"oracle stopped after {ref.iters} iterations (err {ref.err:.3e})")
    res, _ = gpu_solve(prob, k_dtype=torch.float64, check_every=1)
    info = res.info()
    assert info["iters"] == ref.iters
    assert info["err"] <= 1e-6 and not (info["flags"] & uot.UOT_FLAG_NOT_CONVERGED)
    compare(res, ref, 1e-12, 1e-12, "tol stop FP64")
    # coarser checks stop at the first multiple of check_every at or after it
    res7, _ = gpu_solve(prob, k_dtype=torch.float64, check_every=7)
    it7 = res7.info()["iters"]
    assert it7 >= ref.iters and it7 - ref.iters < 7
    ref7 = _oracle(prob, max_iter=it7, tol=0.0)
    compare(res7, ref7, 1e-12, 1e-12, "tol stop, check every 7")


def test_not_converged_flag():
    prob = workloads.headline(n=200, m=300, max_iter=5, tol=1e-12)
    res, _ = gpu_solve(prob, k_dtype=torch.float32)
    info = res.info()
    assert info["iters"] == 5 and (info["flags"] & uot.UOT_FLAG_NOT_CONVERGED)


def test_zero_mass_entries():
    prob = workloads.headline(n=500, m=700, max_iter=25)
    prob.a[[0, 17, 499]] = 0.0
    prob.b[[3, 650]] = 0.0
    ref = _oracle(prob)
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-6)):
        res, _ = gpu_solve(prob, k_dtype=dtype)
        u = res.u.cpu().numpy()
        v = res.v.cpu().numpy()
        assert u[0] == 0 and u[17] == 0 and u[499] == 0 and v[3] == 0 and v[650] == 0
        assert res.info()["flags"] == 0
        compare(res, ref, tol, tol, f"zero mass {dtype}")


def test_zero_iterations():
    prob = workloads.headline(n=300, m=200, max_iter=0)
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float64)
    assert np.all(res.u.cpu().numpy() == 1.0) and np.all(res.v.cpu().numpy() == 1.0)
    assert res.info()["iters"] == 0
    compare(res, ref, 0.0, 1e-12, "max_iter=0")


def test_balanced_limit():
    prob = workloads.headline(n=400, m=640, max_iter=40)
    prob.tau = math.inf
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float64)
    compare(res, ref, 1e-12, 1e-12, "tau=inf")
    c = res.c.cpu().numpy()
    np.testing.assert_allclose(c, prob.b, rtol=1e-13)


def test_underflowing_row_is_flagged():
    prob = workloads.headline(n=64, m=128, max_iter=3)
    C = gpu_cost(prob)
    C[5, :] = 1e4          # exp(-C/eps) underflows to 0 for the whole row
    res, _ = gpu_solve(prob, k_dtype=torch.float32, C=C)
    flags = res.info()["flags"]
    assert flags & uot.UOT_FLAG_ZERO_SUM and flags & uot.UOT_FLAG_NONFINITE


def test_fp32_subnormal_kernel_is_flagged():
    """A 1 x 1 headline problem has K = e^-100, subnormal in FP32: the row
    sum vanishes in FP32 arithmetic and the solve must say so."""
    prob = workloads.headline(n=1, m=1, max_iter=3)
    res, _ = gpu_solve(prob, k_dtype=torch.float32)
    flags = res.info()["flags"]
    assert flags & uot.UOT_FLAG_NONFINITE


def test_warm_start_resume_is_bitwise():
    prob = workloads.headline(n=800, m=1200, max_iter=30)
    C = gpu_cost(prob)
    K = uot.kernel_from_cost(C, prob.eps, torch.float32)
    a, b = to_dev(prob.a), to_dev(prob.b)
    full = uot.sinkhorn(a, b, K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=30)
    first = uot.sinkhorn(a, b, K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=12)
    rest = uot.sinkhorn(a, b, K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=18, v0=first.v)
    torch.cuda.synchronize()
    assert torch.equal(full.u, rest.u) and torch.equal(full.v, rest.v)


def test_bitwise_reproducible():
    prob = workloads.headline(n=3000, m=5000, max_iter=20)
    r1, K = gpu_solve(prob)
    r2, _ = gpu_solve(prob, K=K)
    assert torch.equal(r1.u, r2.u) and torch.equal(r1.v, r2.v) and torch.equal(r1.loss, r2.loss)


def test_argument_errors():
    a = torch.ones(4, dtype=torch.float64, device="cuda")
    b = torch.ones(6, dtype=torch.float64, device="cuda")
    K = torch.ones((4, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, b, K, eps=0.0, tau=1.0, max_iter=3)
    assert e.value.status == 1
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, b, K, eps=0.1, tau=-1.0, max_iter=3)
    assert e.value.status == 1
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, b, K, eps=0.1, tau=1.0, max_iter=-1)
    assert e.value.status == 1
    Kodd = torch.ones((4, 63), dtype=torch.float32, device="cuda")
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, b, Kodd, eps=0.1, tau=1.0, max_iter=3)
    assert e.value.status == 3
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, b, K, eps=0.1, tau=1.0, max_iter=3, tune=99)
    assert e.value.status == 1
    big = torch.ones(20000, dtype=torch.float64, device="cuda")
    Kbig = torch.ones((4, 20032), dtype=torch.float32, device="cuda")
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(a, big, Kbig, eps=0.1, tau=1.0, max_iter=3)
    assert e.value.status == 5


# ------------------------------------------------------------------ full-size checks
def test_rank1_closed_form_full_size():
    """16384 x 16384 FP32, 1000 iterations against the separable-cost closed form."""
    prob = workloads.rank1(16384, 16384, max_iter=1000)
    say("rank-1 16384^2 FP32, 1000 iterations")
    res, _ = gpu_solve(prob, k_dtype=torch.float32)
    lu, lv = pins.rank1(prob.alpha, prob.beta, prob.a, prob.b, prob.eps, prob.tau, 1000)
    eu = float(np.max(np.abs(np.expm1(np.log(res.u.cpu().numpy()) - lu))))
    ev = float(np.max(np.abs(np.expm1(np.log(res.v.cpu().numpy()) - lv))))
    say(f"  err u {eu:.3e} v {ev:.3e}")
    assert eu < 1e-6 and ev < 1e-6


def test_headline_full_size_against_oracle():
    """16384 x 16384 FP32 (the benchmark's launch shape) for 10 iterations,
    element by element against the FP64 oracle run at full size."""
    prob = workloads.headline(max_iter=10)
    say("headline 16384^2, 10 iterations: oracle on the host ...")
    ref = _oracle(prob)
    say("  GPU ...")
    res, _ = gpu_solve(prob, k_dtype=torch.float32)
    compare(res, ref, 1e-6, 1e-6, "headline T=10")


# ------------------------------------------------------------------ persistent loop
@pytest.mark.parametrize("n,m,dtype,tune", [(3000, 5000, torch.float32, 0), (3000, 5000, torch.float64, 0),
                                            (1000, 16381, torch.float32, 6), (2048, 16381, torch.float32, 8),
                                            (257, 100, torch.float32, 0)])
def test_persistent_loop_matches_oracle(n, m, dtype, tune):
    prob = workloads.headline(n=n, m=m, max_iter=25)
    ref = _oracle(prob)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    say(f"persistent n={n} m={m} {dtype} tune={tune}")
    res, _ = gpu_solve(prob, k_dtype=dtype, persistent=True, tune=tune)
    info = res.info()
    assert info["iters"] == 25 and info["flags"] == 0, info
    compare(res, ref, tol, tol, "persistent")


def test_persistent_tolerance_stop():
    prob = workloads.headline(n=900, m=1100, max_iter=2000, tol=1e-6)
    ref = _oracle(prob)
    res, _ = gpu_solve(prob, k_dtype=torch.float64, persistent=True)
    info = res.info()
    assert info["iters"] == ref.iters and info["err"] <= 1e-6
    compare(res, ref, 1e-12, 1e-12, "persistent tol stop")


def test_persistent_headline_full_size():
    prob = workloads.headline(max_iter=10)
    ref = _oracle(prob)
    for tune in (6, 8):
        res, _ = gpu_solve(prob, k_dtype=torch.float32, persistent=True, tune=tune)
        assert res.info()["flags"] == 0
        compare(res, ref, 1e-6, 1e-6, f"persistent headline T=10 tune={tune}")


def test_headline_full_size_tolerance_stop_against_oracle():
    """The headline configuration's own stopping rule at full size: 16384^2
    FP32 K, tol 1e-6 on the relative change of the column marginal, checked
    every iteration; the oracle runs the same rule at full size.  Same
    iteration count, and u, v, loss within 1e-6."""
    prob = workloads.headline(max_iter=2000, tol=1e-6)
    say("headline 16384^2, tol 1e-6: oracle on the host ...")
    ref = _oracle(prob)
    say(f"  oracle stopped after {ref.iters} iterations (err {ref.err:.3e}); GPU ...")
    assert 10 < ref.iters < 2000
    res, _ = gpu_solve(prob, k_dtype=torch.float32)
    info = res.info()
    say(f"  GPU stopped after {info['iters']} iterations (err {info['err']:.3e})")
    assert info["iters"] == ref.iters and info["flags"] == 0
    compare(res, ref, 1e-6, 1e-6, "headline tol stop")


@pytest.mark.parametrize("dtype,m", [(torch.float32, 16381), (torch.float32, 8000), (torch.bfloat16, 8000),
                                     (torch.float8_e4m3fn, 8000), (torch.float64, 3001)])
def test_rows_past_the_last_row_read_zero(dtype, m):
    """K given as the first n rows of a larger allocation whose further rows
    are NaN: the last strip's prefetched rows (and a partial row batch) lie
    past row n and must read as 0, so the result equals the one with K
    alone, bit for bit.  Every read stays inside the allocation."""
    n = 1001
    prob = workloads.precision(n=n, m=m, max_iter=12)
    prob.eps = 0.1            # every entry of exp(-C/eps) >= e^-10: no FP8 row flushes to 0
    C = gpu_cost(prob)
    K = uot.kernel_from_cost(C, prob.eps, dtype)
    ldk = K.shape[1]
    big = torch.empty((n + 64, ldk), dtype=dtype, device="cuda")
    big[:n] = K
    if dtype == torch.float8_e4m3fn:
        big[n:].view(torch.uint8).fill_(0x7F)          # E4M3FN NaN
    else:
        big[n:] = float("nan")
    a, b = to_dev(prob.a), to_dev(prob.b)
    say(f"rows past the end: {dtype} n={n} m={m}")
    r0 = uot.sinkhorn(a, b, K, m=m, eps=prob.eps, tau=prob.tau, max_iter=12)
    r1 = uot.sinkhorn(a, b, big[:n], m=m, eps=prob.eps, tau=prob.tau, max_iter=12)
    torch.cuda.synchronize()
    assert r1.info()["flags"] == 0
    for x, y in ((r0.u, r1.u), (r0.v, r1.v), (r0.r, r1.r), (r0.c, r1.c)):
        assert torch.equal(x, y)
    assert float(r0.loss) == float(r1.loss) and math.isfinite(float(r1.loss))
