"""Batched problems of uneven size in one persistent launch, against the
oracle run on each problem alone (each batch item is an independent
application of the loop).

The batched kernel computes in FP64 on the widened stored K, so with the
stored K handed to both sides (the oracle's FP32 rounding of its own FP64
kernel, uploaded), every problem must match the oracle's FP64 iteration on
those values to 1e-10 (summation order only).  End to end (cost and kernel
built on the GPU), the FP32 bar 1e-6 applies."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import rel_err, say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402


def _oracle_kernel(p, storage):
    C = oracle.cost_points(p.x, p.y, p.cost_kind, p.normalize_max)
    K = oracle.kernel(C, p.eps)
    return K if storage is None else oracle.round_storage(K, storage)


def _stored_on_gpu(K, dtype):
    n, m = K.shape
    ldk = (m + 63) // 64 * 64
    Kp = np.zeros((n, ldk))
    Kp[:, :m] = K
    return torch.from_numpy(Kp).to("cuda").to(dtype)


def _check_against_oracle(res, probs, Ks, bar, tol=0.0, label=""):
    worst = 0.0
    for i, p in enumerate(probs):
        ref = oracle.sinkhorn(Ks[i], p.a, p.b, p.eps, p.tau, p.max_iter, tol)
        u, v, r, c = (t.cpu().numpy() for t in res.problem(i))
        info = res.info(i)
        e = max(rel_err(u, ref.u), rel_err(v, ref.v), rel_err(r, ref.r), rel_err(c, ref.c),
                abs(float(res.loss[i].cpu()) - ref.loss) / abs(ref.loss))
        worst = max(worst, e)
        assert info["iters"] == ref.iters, (i, info, ref.iters)
        assert info["flags"] == 0, (i, info)
        assert e <= bar, (label, i, p.n, p.m, e)
    say(f"  {label}: {len(probs)} problems, worst relative error {worst:.3e}")


def _sizes_problems(ns, ms, seed=3, eps=0.05, tau=1.0, T=60):
    rng = np.random.default_rng(seed)
    probs = []
    for k, (n, m) in enumerate(zip(ns, ms)):
        x = rng.standard_normal((n, 20))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        y = rng.standard_normal((m, 20))
        y /= np.linalg.norm(y, axis=1, keepdims=True)
        a = rng.dirichlet(0.5 * np.ones(n))
        b = rng.dirichlet(0.5 * np.ones(m))
        probs.append(workloads.Problem(f"sz{k}", x, y, a, b, eps=eps, tau=tau, max_iter=T,
                                       cost_kind=workloads.COST_COSINE))
    return probs


# every column-count bucket, ragged tails, single rows and columns
NS = [1, 7, 64, 300, 129, 1000, 33, 2048, 517, 5, 1500, 2]
MS = [1, 16, 100, 256, 257, 512, 700, 1024, 1025, 1500, 2047, 2048]


@pytest.mark.parametrize("dtype,storage", [(torch.float32, "f32"), (torch.float64, None),
                                           (torch.bfloat16, "bf16")])
def test_batched_matches_oracle_on_stored_kernel(dtype, storage):
    probs = _sizes_problems(NS, MS)
    Kr = [_oracle_kernel(p, storage) for p in probs]
    Ks = [_stored_on_gpu(K, dtype) for K in Kr]
    res = uot.sinkhorn_batched(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=[p.eps for p in probs], tau=[p.tau for p in probs], max_iter=60)
    torch.cuda.synchronize()
    _check_against_oracle(res, probs, Kr, 1e-10, label=str(dtype))


def test_batched_tuned_shapes_and_per_problem_parameters():
    """Autotuned tile shapes, per-problem eps and tau (incl. tau = inf)."""
    probs = _sizes_problems(NS, MS, seed=4)
    for k, p in enumerate(probs):
        p.eps = [0.05, 0.1, 0.02][k % 3]
        p.tau = [1.0, float("inf"), 0.3][k % 3]
    Kr = [_oracle_kernel(p, "f32") for p in probs]
    Ks = [_stored_on_gpu(K, torch.float32) for K in Kr]
    solver = uot.BatchedSolver(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=[p.eps for p in probs], tau=[p.tau for p in probs], max_iter=60, tune=1)
    solver.run()
    torch.cuda.synchronize()
    say(f"  shapes {solver.shapes()}")
    _check_against_oracle(solver.result(), probs, Kr, 1e-10, label="tuned")


def test_batched_tolerance_stop_matches_oracle_iterations():
    probs = _sizes_problems(NS[:8], MS[:8], seed=5, T=400)
    Kr = [_oracle_kernel(p, "f32") for p in probs]
    Ks = [_stored_on_gpu(K, torch.float32) for K in Kr]
    res = uot.sinkhorn_batched(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=400, tol=1e-7)
    torch.cuda.synchronize()
    _check_against_oracle(res, probs, Kr, 1e-9, tol=1e-7, label="tol")
    assert any(res.info(i)["iters"] < 400 for i in range(len(probs)))


def test_batched_split_problems_match_oracle():
    """Problems far above the average work per workgroup are split by rows
    over several workgroups, whose parts exchange column sums every
    iteration; the results are still the FP64 iteration on the stored
    kernel (fixed count and tolerance stop), and a small problem is not
    split."""
    probs = _sizes_problems([1800, 900, 40, 2048], [1900, 1100, 30, 64], seed=9, T=80)
    Kr = [_oracle_kernel(p, "f32") for p in probs]
    Ks = [_stored_on_gpu(K, torch.float32) for K in Kr]
    for tol in (0.0, 1e-5):
        solver = uot.BatchedSolver(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                                   eps=[p.eps for p in probs], tau=[p.tau for p in probs], max_iter=80, tol=tol,
                                   trace=True)
        solver.run()
        torch.cuda.synchronize()
        parts = solver.parts()
        say(f"  tol={tol}: parts {parts}, {solver.items} queue entries")
        assert parts[0] > 1 and parts[1] > 1 and parts[2] == 1 and solver.items == sum(parts)
        _check_against_oracle(solver.result(), probs, Kr, 1e-9 if tol > 0 else 1e-10, tol=tol,
                              label=f"split tol={tol}")


def test_batched_zero_mass_entries():
    probs = _sizes_problems([40, 90], [70, 33], seed=6)
    probs[0].a[3] = 0.0
    probs[1].b[:5] = 0.0
    Kr = [_oracle_kernel(p, "f32") for p in probs]
    Ks = [_stored_on_gpu(K, torch.float32) for K in Kr]
    res = uot.sinkhorn_batched(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=60)
    torch.cuda.synchronize()
    u0 = res.problem(0)[0].cpu().numpy()
    v1 = res.problem(1)[1].cpu().numpy()
    assert u0[3] == 0.0 and np.all(v1[:5] == 0.0)
    _check_against_oracle(res, probs, Kr, 1e-10, label="zero mass")


def test_batched_end_to_end_kernels_built_on_gpu():
    """Cost and FP32 kernel built by the library per problem, against the
    oracle's FP64 kernel (FP32 storage error included)."""
    probs = workloads.batched(count=24, lo=16, hi=900, max_iter=100)
    Ks = []
    for p in probs:
        C = uot.cost_from_points(to_dev(p.x), to_dev(p.y), p.cost_kind, p.normalize_max)
        Ks.append(uot.kernel_from_cost(C, p.eps, torch.float32))
    res = uot.sinkhorn_batched(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=100)
    torch.cuda.synchronize()
    _check_against_oracle(res, probs, [_oracle_kernel(p, None) for p in probs], 1e-6, label="end to end")


def test_batched_graph_replays_match_eager():
    probs = _sizes_problems(NS, MS, seed=7, T=40)
    Ks = [_stored_on_gpu(_oracle_kernel(p, "f32"), torch.float32) for p in probs]
    solver = uot.BatchedSolver(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=40)
    solver.run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (solver.u, solver.v, solver.r, solver.c, solver.loss)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        solver.run()                  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solver.run()
    for rep in range(3):
        for t in (solver.u, solver.v, solver.r, solver.c, solver.loss):
            t.fill_(-1.0)             # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, e in zip((solver.u, solver.v, solver.r, solver.c, solver.loss), eager):
            assert torch.equal(t, e), rep


def test_batched_is_bitwise_reproducible_and_traced():
    probs = _sizes_problems(NS, MS, seed=8, T=30)
    Ks = [_stored_on_gpu(_oracle_kernel(p, "f32"), torch.float32) for p in probs]
    solver = uot.BatchedSolver(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=30, trace=True)
    solver.run()
    torch.cuda.synchronize()
    first = solver.u.clone(), solver.v.clone(), solver.loss.clone()
    solver.run()
    torch.cuda.synchronize()
    assert torch.equal(first[0], solver.u) and torch.equal(first[1], solver.v) and torch.equal(first[2], solver.loss)
    t = solver.trace.cpu().numpy().reshape(-1, 2)
    assert np.all(t[:, 1] >= t[:, 0]) and np.all(t[:, 0] > 0)
    f = solver.tail_idle_fraction()
    assert 0.0 <= f < 1.0


def test_batched_argument_errors():
    probs = _sizes_problems([10, 20], [30, 40], seed=9)
    Kr = [_oracle_kernel(p, "f32") for p in probs]
    a = [to_dev(p.a) for p in probs]
    b = [to_dev(p.b) for p in probs]
    K32 = [_stored_on_gpu(K, torch.float32) for K in Kr]
    mixed = [K32[0], _stored_on_gpu(Kr[1], torch.float64)]
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn_batched(mixed, a, b, eps=0.05, tau=1.0, max_iter=5)
    assert e.value.status == 2
    big = _sizes_problems([4], [2049], seed=10)[0]
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn_batched([_stored_on_gpu(_oracle_kernel(big, "f32"), torch.float32)], [to_dev(big.a)],
                             [to_dev(big.b)], eps=0.05, tau=1.0, max_iter=5)
    assert e.value.status == 5
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn_batched(K32, a, b, eps=-1.0, tau=1.0, max_iter=5)
    assert e.value.status == 1


def test_batched_full_size_sampled():
    """1024 problems, n, m ~ U[16, 2048], 300-D cosine, 200 iterations, FP32
    K built on the GPU; every problem finishes with flags 0 and 200
    iterations; 6 sampled problems (the largest, the smallest and 4 random)
    against the oracle on their own FP32-rounded kernels given to the batch."""
    probs = workloads.batched()
    rng = np.random.default_rng(11)
    work = np.array([p.n * p.m for p in probs])
    sample = sorted({int(np.argmax(work)), int(np.argmin(work)), *rng.choice(len(probs), 4, replace=False).tolist()})
    say(f"  building {len(probs)} kernels on the GPU ...")
    Ks = []
    Kr = {}
    for i, p in enumerate(probs):
        if i in sample:
            Kr[i] = _oracle_kernel(p, "f32")
            Ks.append(_stored_on_gpu(Kr[i], torch.float32))
        else:
            C = uot.cost_from_points(to_dev(p.x), to_dev(p.y), p.cost_kind, p.normalize_max)
            Ks.append(uot.kernel_from_cost(C, p.eps, torch.float32))
            del C
    say("  solving ...")
    res = uot.sinkhorn_batched(Ks, [to_dev(p.a) for p in probs], [to_dev(p.b) for p in probs],
                               eps=0.05, tau=1.0, max_iter=200)
    torch.cuda.synchronize()
    info = np.frombuffer(res.info_raw.cpu().numpy().tobytes(), dtype=np.uint8).reshape(len(probs), -1)
    infos = [_lib_info(row) for row in info]
    assert all(x[0] == 200 and x[3] == 0 for x in infos)
    assert torch.isfinite(res.loss).all()
    _check_against_oracle(_subset(res, sample), [probs[i] for i in sample], [Kr[i] for i in sample], 1e-10,
                          label="full size, sampled")


def _lib_info(raw):
    from paper_2412_11079_amd import _lib
    s = _lib.Info.from_buffer_copy(bytes(raw))
    return s.iters, s.err, s.absorptions, s.flags


class _subset:
    def __init__(self, res, idx):
        self.res, self.idx = res, idx
        self.loss = res.loss[idx]

    def problem(self, k):
        return self.res.problem(self.idx[k])

    def info(self, k):
        return self.res.info(self.idx[k])
