"""The paper's literal in-place matrix rescaling (Section 2.1 in the
single-pass order of Section 4.1's Algorithm 1) on the GPU against the
oracle's transcription of the same steps."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import gpu_cost, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


def _run(prob, dtype, T, tol=0.0, check_every=1, tune=0):
    K = uot.kernel_from_cost(gpu_cost(prob), prob.eps, dtype)
    A = K.clone()
    res = uot.matrix_rescale_(A, to_dev(prob.a), to_dev(prob.b), m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=T,
                              tol=tol, check_every=check_every, tune=tune)
    torch.cuda.synchronize()
    return K, A, res


def _errors(got, ref):
    """(entrywise relative error over entries in the full-precision FP32
    range, >= 2^-100, and the normwise relative error).  Smaller entries of
    an FP32 matrix lose relative precision as the rescaling moves them
    through the subnormal range; their share of the matrix's mass is below
    2^-100 relative."""
    big = np.abs(ref) >= 2.0 ** -100
    e = rel_err(got[big], ref[big])
    nrm = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return e, nrm


def _oracle(prob, K, T):
    Kr = K[:, :prob.m].cpu().double().numpy()   # the stored start matrix (the oracle rescales the same values)
    return oracle.matrix_rescale(Kr, prob.a, prob.b, prob.eps, prob.tau, T)


@pytest.mark.parametrize("n,m,dtype,T,tol", [
    (300, 257, torch.float64, 20, 1e-11), (1001, 1531, torch.float64, 15, 1e-11), (257, 100, torch.float64, 30, 1e-11),
    (300, 257, torch.float32, 20, 2e-5), (1001, 1531, torch.float32, 15, 2e-5), (2000, 16381, torch.float32, 5, 2e-5)])
def test_matrix_rescale_matches_oracle(n, m, dtype, T, tol):
    prob = workloads.headline(n=n, m=m, max_iter=T)
    say(f"in-place form {dtype} n={n} m={m} T={T}")
    K, A, res = _run(prob, dtype, T)
    ref, r0, c0 = _oracle(prob, K, T)
    got = A[:, :m].cpu().double().numpy()
    e, nrm = _errors(got, ref)
    er = rel_err(res.r.cpu().numpy(), r0)
    ec = rel_err(res.c.cpu().numpy(), c0)
    say(f"  A {e:.3e} (normwise {nrm:.3e})  row sums {er:.3e}  column sums {ec:.3e}")
    info = res.info()
    assert info["iters"] == T and info["flags"] == 0
    assert e <= tol and nrm <= tol and er <= tol and ec <= tol
    if dtype == torch.float64:
        assert rel_err(got, ref) <= tol
    assert torch.all(A[:, m:] == 0)          # padding columns hold 0


def test_matrix_rescale_tolerance_stop_equals_fixed_count():
    prob = workloads.headline(n=900, m=1100, max_iter=3000)
    _, A1, r1 = _run(prob, torch.float64, 3000, tol=1e-9, check_every=4)
    it = r1.info()["iters"]
    say(f"  tolerance 1e-9 stopped after {it} iterations")
    assert 1 < it < 3000 and r1.info()["err"] <= 1e-9
    _, A2, r2 = _run(prob, torch.float64, it)
    assert torch.equal(A1, A2) and torch.equal(r1.beta, r2.beta)


def test_matrix_rescale_every_one_row_shape():
    prob = workloads.headline(n=513, m=500, max_iter=6)          # every one-row shape covers 500 FP64 columns
    base = None
    for tune in range(1, 9):
        K, A, res = _run(prob, torch.float64, 6, tune=tune)
        if base is None:
            ref, _, _ = _oracle(prob, K, 6)
            base = ref
        assert rel_err(A[:, :prob.m].cpu().numpy(), base) <= 1e-11, tune


def test_matrix_rescale_argument_errors():
    prob = workloads.headline(n=64, m=64, max_iter=3)
    K = uot.kernel_from_cost(gpu_cost(prob), prob.eps, torch.bfloat16)
    with pytest.raises(ValueError):
        uot.matrix_rescale_(K, to_dev(prob.a), to_dev(prob.b), eps=prob.eps, tau=prob.tau, max_iter=3)
    K = uot.kernel_from_cost(gpu_cost(prob), prob.eps, torch.float32)
    with pytest.raises(uot.UOTError) as e:            # the in-place form runs the one-row shapes 1-8
        uot.matrix_rescale_(K, to_dev(prob.a), to_dev(prob.b), eps=prob.eps, tau=prob.tau, max_iter=3, tune=9)
    assert e.value.status == 5


def test_matrix_rescale_full_size():
    """16384^2 FP32 (the headline matrix), 10 iterations, against the oracle
    at full size: row and column sums, both factor vectors, and 64 sampled
    rows of the rescaled matrix."""
    prob = workloads.headline(max_iter=10)
    say("in-place form at 16384^2: GPU ...")
    K, A, res = _run(prob, torch.float32, 10)
    say("  oracle on the host ...")
    ref, r0, c0 = _oracle(prob, K, 10)
    rows = np.sort(np.random.default_rng(3).choice(prob.n, 64, replace=False))
    e, nrm = _errors(A[rows, :prob.m].cpu().double().numpy(), ref[rows])
    er = rel_err(res.r.cpu().numpy(), r0)
    ec = rel_err(res.c.cpu().numpy(), c0)
    say(f"  sampled rows {e:.3e} (normwise {nrm:.3e})  row sums {er:.3e}  column sums {ec:.3e}")
    assert res.info()["flags"] == 0
    assert e <= 2e-5 and nrm <= 2e-5 and er <= 2e-5 and ec <= 2e-5
