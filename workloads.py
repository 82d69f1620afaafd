"""Seeded synthetic inputs for the entropic UOT Sinkhorn loop.

This module is shared by the FP64 CPU oracle (via the tests and the bench's
CPU leg) and by the HIP path (via the tests, the bench and the smoke run).
It draws points and histograms only: it computes no cost, no kernel and no
Sinkhorn arithmetic, so that the two implementations under test share no
part of the method.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) in FP64 and
draws in the fixed order: sizes, source points ``x``, target points ``y``,
source histogram ``a``, target histogram ``b``.  The sizes can be reduced
for parity tests; the recipe (distribution, structure, parameters) stays the
one of the named workload.

Workloads (problem statement: Section 2.1; the paper's own data are its
colour-transfer images and unnamed dense matrices, which these stand in for):

* ``plain_fp64``   2-D points uniform in [0,1]^2, squared-Euclidean cost,
                   ``a`` uniform-random positive normalised to 1, ``b`` to 1.3,
                   eps=0.05, tau=1, exactly 100 iterations.       N=M=1024.
* ``headline``     3-D points from an 8-component Gaussian mixture
                   (sigma 0.1, means uniform in [0,1]^3, equal weights),
                   squared-Euclidean cost divided by its maximum,
                   a ~ Dirichlet(1), b ~ 0.8 Dirichlet(1), eps=0.01, tau=0.5,
                   1000 iterations (or tol 1e-6 on the column-marginal change).
                   N=M=16384.
* ``precision``    16-D standard-normal points, squared-Euclidean / max,
                   a, b ~ Dirichlet(1), eps=1e-3, tau=0.1, 2000 iterations,
                   absorption when |log u| or |log v| exceeds 30.
                   N=65536, M=8192.
* ``batched``      1024 problems with n, m uniform in [16, 2048], 300-D unit
                   embeddings, cosine cost 1 - x.y, Dirichlet(0.5)
                   histograms, eps=0.05, tau=1, 200 iterations.
* ``multi_rhs``    one shared 8192 x 8192 cosine kernel (300-D unit rows) and
                   256 Dirichlet(0.5) histogram pairs.
* ``grad``         3-D points uniform in the unit cube, target shifted by
                   0.2, uniform histograms, squared-Euclidean cost (not
                   normalised), eps=0.02, tau=1, 500 iterations, checkpoints
                   every 50.  N=M=8192.
* ``rank1``        separable cost C_ij = alpha_i + beta_j (closed-form pin).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

COST_SQEUCLID = 0
COST_COSINE = 1

SEEDS = {"plain_fp64": 1, "headline": 2, "precision": 3, "batched": 4,
         "grad": 5, "multi_rhs": 6, "rank1": 101}


@dataclass
class Problem:
    """One UOT problem: points (or a separable cost), histograms, parameters."""
    name: str
    x: Optional[np.ndarray]          # (n, d) float64 source points, or None
    y: Optional[np.ndarray]          # (m, d) float64 target points, or None
    a: np.ndarray                    # (n,) float64 >= 0
    b: np.ndarray                    # (m,) float64 >= 0
    eps: float
    tau: float                       # math.inf means balanced (fi = 1)
    max_iter: int
    tol: float = 0.0
    cost_kind: int = COST_SQEUCLID
    normalize_max: bool = False
    absorb_log_threshold: float = 0.0
    checkpoint_every: int = 0
    alpha: Optional[np.ndarray] = None   # separable cost only
    beta: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.a.shape[0])

    @property
    def m(self) -> int:
        return int(self.b.shape[0])


def _uniform_positive(rng, k):
    # 1 - U[0,1) lies in (0, 1]: strictly positive weights.
    return 1.0 - rng.random(k)


def plain_fp64(n: int = 1024, m: int = 1024, seed: int = SEEDS["plain_fp64"]) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2))
    y = rng.random((m, 2))
    a = _uniform_positive(rng, n)
    a = a / a.sum()
    b = _uniform_positive(rng, m)
    b = 1.3 * (b / b.sum())
    return Problem("plain_fp64", x, y, a, b, eps=0.05, tau=1.0, max_iter=100,
                   cost_kind=COST_SQEUCLID, normalize_max=False)


def _gmm_points(rng, means, k, sigma):
    comp = rng.integers(0, means.shape[0], k)
    return means[comp] + sigma * rng.standard_normal((k, means.shape[1]))


def headline(n: int = 16384, m: int = 16384, seed: int = SEEDS["headline"],
             max_iter: int = 1000, tol: float = 0.0) -> Problem:
    rng = np.random.default_rng(seed)
    means = rng.random((8, 3))
    x = _gmm_points(rng, means, n, 0.1)
    y = _gmm_points(rng, means, m, 0.1)
    a = rng.dirichlet(np.ones(n))
    b = 0.8 * rng.dirichlet(np.ones(m))
    return Problem("headline", x, y, a, b, eps=0.01, tau=0.5, max_iter=max_iter,
                   tol=tol, cost_kind=COST_SQEUCLID, normalize_max=True)


def precision(n: int = 65536, m: int = 8192, seed: int = SEEDS["precision"],
              max_iter: int = 2000) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 16))
    y = rng.standard_normal((m, 16))
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    return Problem("precision", x, y, a, b, eps=1e-3, tau=0.1, max_iter=max_iter,
                   cost_kind=COST_SQEUCLID, normalize_max=True,
                   absorb_log_threshold=30.0)


def _unit_rows(rng, k, d):
    z = rng.standard_normal((k, d))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


def batched(count: int = 1024, lo: int = 16, hi: int = 2048, d: int = 300,
            seed: int = SEEDS["batched"], max_iter: int = 200) -> list:
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, count)
    ms = rng.integers(lo, hi + 1, count)
    probs = []
    for p in range(count):
        x = _unit_rows(rng, int(ns[p]), d)
        y = _unit_rows(rng, int(ms[p]), d)
        a = rng.dirichlet(0.5 * np.ones(int(ns[p])))
        b = rng.dirichlet(0.5 * np.ones(int(ms[p])))
        probs.append(Problem(f"batched[{p}]", x, y, a, b, eps=0.05, tau=1.0,
                             max_iter=max_iter, cost_kind=COST_COSINE))
    return probs


def multi_rhs(n: int = 8192, m: int = 8192, R: int = 256, d: int = 300,
              seed: int = SEEDS["multi_rhs"], max_iter: int = 200):
    """Shared cosine kernel with R histogram pairs; returns (Problem, A, B)."""
    rng = np.random.default_rng(seed)
    x = _unit_rows(rng, n, d)
    y = _unit_rows(rng, m, d)
    A = rng.dirichlet(0.5 * np.ones(n), size=R).T.copy()   # (n, R)
    B = rng.dirichlet(0.5 * np.ones(m), size=R).T.copy()   # (m, R)
    base = Problem("multi_rhs", x, y, A[:, 0].copy(), B[:, 0].copy(), eps=0.05,
                   tau=1.0, max_iter=max_iter, cost_kind=COST_COSINE)
    return base, A, B


def grad(n: int = 8192, m: int = 8192, seed: int = SEEDS["grad"],
         max_iter: int = 500) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    y = rng.random((m, 3)) + 0.2
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    return Problem("grad", x, y, a, b, eps=0.02, tau=1.0, max_iter=max_iter,
                   cost_kind=COST_SQEUCLID, normalize_max=False,
                   checkpoint_every=50)


def rank1(n: int, m: int, seed: int = SEEDS["rank1"], eps: float = 0.05,
          tau: float = 0.5, max_iter: int = 50) -> Problem:
    """Separable cost C_ij = alpha_i + beta_j with alpha, beta in [0, 1).

    With eps = 0.05 every kernel entry exp(-C/eps) >= e^-40 stays a normal
    FP32 number, so FP32 storage only rounds it."""
    rng = np.random.default_rng(seed)
    alpha = rng.random(n)
    beta = rng.random(m)
    a = rng.dirichlet(np.ones(n))
    b = 0.8 * rng.dirichlet(np.ones(m))
    return Problem("rank1", None, None, a, b, eps=eps, tau=tau, max_iter=max_iter,
                   alpha=alpha, beta=beta)


def random_small(n: int, m: int, seed: int, eps: float = 0.1, tau: float = 1.0,
                 d: int = 2, max_iter: int = 50) -> Problem:
    """Generic small problem (uniform points, Dirichlet(1) histograms)."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    y = rng.random((m, d))
    a = rng.dirichlet(np.ones(n))
    b = 1.1 * rng.dirichlet(np.ones(m))
    return Problem("random_small", x, y, a, b, eps=eps, tau=tau, max_iter=max_iter)

