"""Pins of the FP64 oracle against mathematics that fixes its results.

Every test here runs on the CPU.  The oracle is exercised on rectangular
(n != m), non-symmetric problems so that a transposed operand, a swapped
index, a dropped term or a wrong sign in it fails at least one test.
"""
import math

import numpy as np
import pytest

import oracle
import pins
import workloads


def _problem_arrays(prob):
    C = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    K = oracle.kernel(C, prob.eps)
    return C, K


# ---------------------------------------------------------------- P1: 1 x 1
@pytest.mark.parametrize("T", [1, 2, 3, 7, 40])
@pytest.mark.parametrize("tau", [1.0, 0.3, math.inf])
def test_one_by_one_iterates(T, tau):
    a, b, C, eps = 0.7, 1.3, 0.4, 0.05
    K = np.array([[math.exp(-C / eps)]])
    res = oracle.sinkhorn(K, np.array([a]), np.array([b]), eps, tau, T)
    u_ref, v_ref = pins.one_by_one(a, b, C, eps, tau, T)
    assert res.iters == T
    assert res.u[0] == pytest.approx(u_ref, rel=1e-13)
    assert res.v[0] == pytest.approx(v_ref, rel=1e-13)


def test_one_by_one_limit_and_counterexample():
    # Vector form reaches the UOT optimum; the paper's literal in-place form
    # with fi < 1 reaches a different, cost-independent value (a reading
    # recorded in the design notes).
    a, b, C, eps, tau = 0.7, 1.3, 0.4, 0.05, 1.0
    K = np.array([[math.exp(-C / eps)]])
    res = oracle.sinkhorn(K, np.array([a]), np.array([b]), eps, tau, 2000)
    P = res.u[0] * K[0, 0] * res.v[0]
    assert P == pytest.approx(pins.one_by_one_limit(a, b, C, eps, tau), rel=1e-13)
    assert P == pytest.approx(0.785742, abs=5e-7)
    A = pins.paper_matrix_form(K, np.array([a]), np.array([b]), eps, tau, 2000)
    fi = pins.fi_of(eps, tau)
    literal = math.exp((math.log(b) + (1 - fi) * math.log(a)) / (2 - fi))
    assert A[0, 0] == pytest.approx(literal, rel=1e-12)
    assert A[0, 0] == pytest.approx(1.26393, abs=5e-6)


# ---------------------------------------------------------------- P2: rank 1
@pytest.mark.parametrize("n,m,T", [(37, 53, 1), (37, 53, 5), (64, 19, 30), (200, 311, 60)])
@pytest.mark.parametrize("tau", [0.5, math.inf])
def test_rank1_closed_form(n, m, T, tau):
    prob = workloads.rank1(n, m, tau=tau)
    C = np.add.outer(prob.alpha, prob.beta)
    K = oracle.kernel(C, prob.eps)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T)
    lu, lv = pins.rank1(prob.alpha, prob.beta, prob.a, prob.b, prob.eps, prob.tau, T)
    np.testing.assert_allclose(np.log(res.u), lu, rtol=0, atol=1e-11)
    np.testing.assert_allclose(np.log(res.v), lv, rtol=0, atol=1e-11)


# ---------------------------------------------------------------- P3: balanced limit
def test_balanced_column_marginal_exact_and_paper_form():
    prob = workloads.random_small(23, 17, seed=7, eps=0.2, tau=math.inf)
    C, K = _problem_arrays(prob)
    for T in (1, 4, 25):
        res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, math.inf, T)
        # after each column half-step with fi = 1 the column marginal is b
        np.testing.assert_allclose(res.c, prob.b, rtol=1e-13, atol=0)
        A = pins.paper_matrix_form(K, prob.a, prob.b, prob.eps, math.inf, T)
        P = res.u[:, None] * K * res.v[None, :]
        np.testing.assert_allclose(P, A, rtol=1e-12, atol=1e-300)


def test_balanced_row_marginal_converges_with_equal_mass():
    prob = workloads.random_small(23, 17, seed=8, eps=0.2, tau=math.inf)
    b = prob.b / prob.b.sum()             # equal masses
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, b, prob.eps, math.inf, 3000)
    np.testing.assert_allclose(res.r, prob.a, rtol=1e-10)


def test_large_tau_approaches_balanced():
    prob = workloads.random_small(15, 21, seed=9, eps=0.2, tau=math.inf)
    b = prob.b / prob.b.sum()
    C, K = _problem_arrays(prob)
    bal = oracle.sinkhorn(K, prob.a, b, prob.eps, math.inf, 3000)
    unb = oracle.sinkhorn(K, prob.a, b, prob.eps, 1e6, 3000)
    P0 = bal.u[:, None] * K * bal.v[None, :]
    P1 = unb.u[:, None] * K * unb.v[None, :]
    assert np.max(np.abs(P1 - P0)) / np.max(P0) < 1e-5


# ---------------------------------------------------------------- P4: invariants
def _converged_plan(C, a, b, eps, tau, iters=4000):
    K = oracle.kernel(C, eps)
    res = oracle.sinkhorn(K, a, b, eps, tau, iters)
    return res.u[:, None] * K * res.v[None, :]


def test_cost_shift_and_mass_scaling_invariants():
    prob = workloads.random_small(11, 14, seed=10, eps=0.3, tau=0.7)
    C, _ = _problem_arrays(prob)
    eps, tau = prob.eps, prob.tau
    P = _converged_plan(C, prob.a, prob.b, eps, tau)
    k = 0.37
    Pk = _converged_plan(C + k, prob.a, prob.b, eps, tau)
    np.testing.assert_allclose(Pk, P * math.exp(-k / (eps + 2 * tau)), rtol=1e-11)
    lam = 2.5
    Pl = _converged_plan(C, lam * prob.a, lam * prob.b, eps, tau)
    np.testing.assert_allclose(Pl, P * lam ** (2 * tau / (eps + 2 * tau)), rtol=1e-11)


def test_permutation_equivariance():
    prob = workloads.random_small(12, 9, seed=11, eps=0.1, tau=0.5)
    C, K = _problem_arrays(prob)
    rng = np.random.default_rng(0)
    pi, rho = rng.permutation(12), rng.permutation(9)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 17)
    resp = oracle.sinkhorn(K[pi][:, rho], prob.a[pi], prob.b[rho], prob.eps, prob.tau, 17)
    np.testing.assert_allclose(resp.u, res.u[pi], rtol=1e-13)
    np.testing.assert_allclose(resp.v, res.v[rho], rtol=1e-13)
    assert resp.loss == pytest.approx(res.loss, rel=1e-13)


# ---------------------------------------------------------------- P5: dual ascent
def test_dual_monotone_and_weak_duality():
    prob = workloads.random_small(13, 8, seed=12, eps=0.15, tau=0.8)
    C, K = _problem_arrays(prob)
    T = 60
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T, trace=True)
    tr = res.trace
    eps, tau = prob.eps, prob.tau
    vals = []
    gaps = []
    for t in range(1, T + 1):
        u = tr["u"][t - 1]
        vprev, v = tr["v"][t - 1], tr["v"][t]
        vals.append(pins.dual_value(eps * np.log(u), eps * np.log(vprev), C, prob.a, prob.b, eps, tau))
        vals.append(pins.dual_value(eps * np.log(u), eps * np.log(v), C, prob.a, prob.b, eps, tau))
        P = u[:, None] * K * v[None, :]
        gaps.append(pins.primal_value(P, C, prob.a, prob.b, eps, tau) - vals[-1])
    vals = np.array(vals)
    assert np.all(np.diff(vals) >= -1e-14 * np.abs(vals[1:]))
    assert min(gaps) >= -1e-13
    assert gaps[-1] < 1e-3 * gaps[0]


# ---------------------------------------------------------------- P6: objective identity
@pytest.mark.parametrize("tau", [0.6, math.inf])
def test_loss_identity_equals_definition(tau):
    prob = workloads.random_small(19, 26, seed=13, eps=0.07, tau=tau)
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, tau, 9)
    direct, tc = oracle.loss_direct(C, K, res.u, res.v, prob.a, prob.b, prob.eps, tau)
    P = res.u[:, None] * K * res.v[None, :]
    numpy_def = pins.primal_value(P, C, prob.a, prob.b, prob.eps, tau)
    assert res.loss == pytest.approx(direct, rel=1e-12)
    assert direct == pytest.approx(numpy_def, rel=1e-12)
    assert tc == pytest.approx(float((C * P).sum()), rel=1e-12)


# ---------------------------------------------------------------- P7: Newton dual
@pytest.mark.parametrize("n,m,eps,tau", [(5, 7, 0.5, 1.0), (8, 6, 0.1, 0.4), (3, 8, 0.05, 1.0)])
def test_newton_dual_matches_converged_sinkhorn(n, m, eps, tau):
    prob = workloads.random_small(n, m, seed=14 + n, eps=eps, tau=tau)
    C, K = _problem_arrays(prob)
    u_n, v_n, gnorm = pins.newton_dual(C, prob.a, prob.b, eps, tau)
    assert gnorm < 1e-13
    res = oracle.sinkhorn(K, prob.a, prob.b, eps, tau, 20000)
    P_s = res.u[:, None] * K * res.v[None, :]
    P_n = u_n[:, None] * K * v_n[None, :]
    np.testing.assert_allclose(P_s, P_n, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(res.u, u_n, rtol=1e-10)
    np.testing.assert_allclose(res.v, v_n, rtol=1e-10)


# ---------------------------------------------------------------- P8: fixed point
def test_fixed_point_residual_vanishes():
    prob = workloads.plain_fp64(n=120, m=90)
    C, K = _problem_arrays(prob)
    fi = pins.fi_of(prob.eps, prob.tau)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 3000)
    Kv = K @ res.v
    KTu = K.T @ res.u
    assert np.max(np.abs(np.log(res.u) - fi * (np.log(prob.a) - np.log(Kv)))) < 1e-11
    assert np.max(np.abs(np.log(res.v) - fi * (np.log(prob.b) - np.log(KTu)))) < 1e-11


# ---------------------------------------------------------------- P9: adjoint
def _fd_loss(C, a, b, eps, tau, T):
    K = oracle.kernel(C, eps)
    return oracle.sinkhorn(K, a, b, eps, tau, T).loss


@pytest.mark.parametrize("T", [1, 3, 12])
@pytest.mark.parametrize("tau", [0.8, math.inf])
def test_adjoint_matches_central_differences(T, tau):
    prob = workloads.random_small(6, 5, seed=21, eps=0.2, tau=tau)
    C, K = _problem_arrays(prob)
    a, b, eps = prob.a, prob.b, prob.eps
    res = oracle.sinkhorn(K, a, b, eps, tau, T, trace=True)
    ga, gb, G = oracle.adjoint(K, a, b, eps, tau, res)
    # steps relative to each histogram entry (some are ~1e-4)
    ha = 1e-5 * a
    hb = 1e-5 * b
    fd_a = np.array([(_fd_loss(C, a + ha[i] * e, b, eps, tau, T)
                      - _fd_loss(C, a - ha[i] * e, b, eps, tau, T)) / (2 * ha[i])
                     for i, e in enumerate(np.eye(6))])
    fd_b = np.array([(_fd_loss(C, a, b + hb[j] * e, eps, tau, T)
                      - _fd_loss(C, a, b - hb[j] * e, eps, tau, T)) / (2 * hb[j])
                     for j, e in enumerate(np.eye(5))])
    h = 1e-6
    fd_C = np.zeros_like(C)
    for i in range(6):
        for j in range(5):
            E = np.zeros_like(C)
            E[i, j] = h
            fd_C[i, j] = (_fd_loss(C + E, a, b, eps, tau, T) - _fd_loss(C - E, a, b, eps, tau, T)) / (2 * h)
    scale_a = max(1.0, np.max(np.abs(fd_a)))
    np.testing.assert_allclose(ga, fd_a, rtol=0, atol=2e-7 * scale_a)
    np.testing.assert_allclose(gb, fd_b, rtol=0, atol=2e-7 * max(1.0, np.max(np.abs(fd_b))))
    np.testing.assert_allclose(G, fd_C, rtol=0, atol=2e-7 * max(1.0, np.max(np.abs(fd_C))))


def test_adjoint_points_matches_central_differences():
    prob = workloads.grad(n=7, m=6, max_iter=8)
    eps, tau, T = prob.eps, prob.tau, prob.max_iter

    def loss_x(x):
        C = oracle.cost_points(x, prob.y, 0, False)
        return _fd_loss(C, prob.a, prob.b, eps, tau, T)

    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, eps, tau, T, trace=True)
    _, _, G = oracle.adjoint(K, prob.a, prob.b, eps, tau, res)
    gx = oracle.grad_points_sqeuclid(G, prob.x, prob.y)
    h = 1e-6
    fd = np.zeros_like(prob.x)
    for i in range(prob.x.shape[0]):
        for k in range(3):
            E = np.zeros_like(prob.x)
            E[i, k] = h
            fd[i, k] = (loss_x(prob.x + E) - loss_x(prob.x - E)) / (2 * h)
    np.testing.assert_allclose(gx, fd, rtol=0, atol=2e-7 * max(1.0, np.max(np.abs(fd))))


def test_adjoint_target_points_matches_central_differences():
    """dL/dy from G against central differences of the loss in each target
    coordinate (rectangular: a swapped x/y or a wrong sign fails)."""
    prob = workloads.grad(n=6, m=8, max_iter=7)
    eps, tau, T = prob.eps, prob.tau, prob.max_iter

    def loss_y(y):
        C = oracle.cost_points(prob.x, y, 0, False)
        return _fd_loss(C, prob.a, prob.b, eps, tau, T)

    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, eps, tau, T, trace=True)
    _, _, G = oracle.adjoint(K, prob.a, prob.b, eps, tau, res)
    gy = oracle.grad_target_sqeuclid(G, prob.x, prob.y)
    h = 1e-6
    fd = np.zeros_like(prob.y)
    for j in range(prob.y.shape[0]):
        for k in range(3):
            E = np.zeros_like(prob.y)
            E[j, k] = h
            fd[j, k] = (loss_y(prob.y + E) - loss_y(prob.y - E)) / (2 * h)
    np.testing.assert_allclose(gy, fd, rtol=0, atol=2e-7 * max(1.0, np.max(np.abs(fd))))


def test_potential_marginals_and_loss_match_plain_run():
    """Marginals summed from exp((f+g-C)/eps) equal u (K v) and v (K^T u) of a
    plain run, and the potential form of the objective equals its
    definition summed over the plan."""
    prob = workloads.random_small(13, 9, seed=31, eps=0.07, tau=0.6)
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 25)
    f, g = prob.eps * np.log(res.u), prob.eps * np.log(res.v)
    r, c = oracle.potential_marginals(C, f, g, prob.eps)
    np.testing.assert_allclose(r, res.r, rtol=1e-13)
    np.testing.assert_allclose(c, res.c, rtol=1e-13)
    L_direct, _ = oracle.loss_direct(C, K, res.u, res.v, prob.a, prob.b, prob.eps, prob.tau)
    L = oracle.loss_potentials(f, g, r, c, prob.a, prob.b, prob.eps, prob.tau)
    assert L == pytest.approx(L_direct, rel=1e-12)
    # a zero scaling (f = -inf) removes its row from both marginals
    f2 = f.copy()
    f2[3] = -np.inf
    r2, c2 = oracle.potential_marginals(C, f2, g, prob.eps)
    assert r2[3] == 0.0
    np.testing.assert_allclose(c2, c - np.exp((f[3] + g - C[3]) / prob.eps), rtol=1e-12)


def test_adjoint_envelope_at_convergence():
    # At the optimum dL/dC = P, dL/da = tau (1 - r/a), dL/db = tau (1 - c/b).
    prob = workloads.random_small(9, 7, seed=22, eps=0.3, tau=1.0)
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 400, trace=True)
    ga, gb, G = oracle.adjoint(K, prob.a, prob.b, prob.eps, prob.tau, res)
    P = res.u[:, None] * K * res.v[None, :]
    np.testing.assert_allclose(G, P, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(ga, prob.tau * (1 - res.r / prob.a), rtol=0, atol=1e-9)
    np.testing.assert_allclose(gb, prob.tau * (1 - res.c / prob.b), rtol=0, atol=1e-9)


def test_matrix_rescale_balanced_equals_vector_form():
    """fi = 1 (tau = inf): the literal in-place rescaling after T iterations
    is diag(alpha) K diag(beta) with alpha, beta the vector-form scalings
    taken columns first, i.e. the oracle's rows-first iteration on K^T with
    the histograms swapped."""
    prob = workloads.random_small(11, 7, seed=51, eps=0.2, tau=math.inf)
    C, K = _problem_arrays(prob)
    for T in (1, 2, 9):
        A, r, c = oracle.matrix_rescale(K, prob.a, prob.b, prob.eps, prob.tau, T)
        res = oracle.sinkhorn(K.T.copy(), prob.b, prob.a, prob.eps, prob.tau, T)
        P = (res.u[:, None] * K.T * res.v[None, :]).T
        np.testing.assert_allclose(A, P, rtol=1e-12, atol=0)
        np.testing.assert_allclose(r, A.sum(axis=1), rtol=1e-13)
        np.testing.assert_allclose(c, A.sum(axis=0), rtol=1e-13)
        np.testing.assert_allclose(r, prob.a, rtol=1e-12)         # rows are rescaled last


def test_matrix_rescale_separable_closed_form():
    """A rank-1 start A = k1 k2^T stays rank-1 under the literal rescaling,
    with the O(n + m) recurrence (columns, then rows)
      k2 <- k2^(1-fi) b^fi S1^(-fi),  S1 = sum k1,
      k1 <- k1^(1-fi) a^fi S2^(-fi),  S2 = sum k2,
    checked at every T against the O(nm) in-place rescaling, fi < 1."""
    rng = np.random.default_rng(52)
    n, m = 9, 14
    k1 = np.exp(-rng.random(n))
    k2 = np.exp(-rng.random(m))
    a = 0.5 + rng.random(n)
    b = 0.5 + rng.random(m)
    eps, tau = 0.05, 0.7
    fi = tau / (tau + eps)
    for T in (1, 3, 10):
        A, _, _ = oracle.matrix_rescale(np.outer(k1, k2), a, b, eps, tau, T)
        l1, l2 = np.log(k1), np.log(k2)
        for _ in range(T):
            l2 = (1 - fi) * l2 + fi * np.log(b) - fi * np.log(np.exp(l1).sum())
            l1 = (1 - fi) * l1 + fi * np.log(a) - fi * np.log(np.exp(l2).sum())
        np.testing.assert_allclose(A, np.exp(l1[:, None] + l2[None, :]), rtol=1e-12)


def test_matrix_rescale_one_by_one_limit_is_cost_independent():
    """1 x 1: log A after a column and a row step is (1-fi)^2 log A + (1-fi)
    fi log b + fi log a; the fixed point ((1-fi) log b + log a)/(2 - fi) does
    not depend on the cost, unlike the vector form's optimum."""
    eps, tau, a, b, C = 0.05, 1.0, 0.7, 1.3, 0.4
    fi = tau / (tau + eps)
    K = np.array([[math.exp(-C / eps)]])
    x = math.log(K[0, 0])
    for T in range(1, 6):
        x = (1 - fi) * ((1 - fi) * x + fi * math.log(b)) + fi * math.log(a)
        A, _, _ = oracle.matrix_rescale(K, [a], [b], eps, tau, T)
        assert math.log(A[0, 0]) == pytest.approx(x, abs=1e-13)
    A, _, _ = oracle.matrix_rescale(K, [a], [b], eps, tau, 400)
    assert math.log(A[0, 0]) == pytest.approx(((1 - fi) * math.log(b) + math.log(a)) / (2 - fi), abs=1e-12)


def test_envelope_gradients_equal_unrolled_adjoint_at_convergence():
    """The oracle's implicit gradients against its unrolled reverse mode
    (pinned by finite differences) once the iterates have converged
    (fi^(2T) ~ 1e-35 here), on a rectangular problem with both histograms
    unnormalised; and the point gradients built from them."""
    prob = workloads.random_small(13, 8, seed=41, eps=0.25, tau=0.7)
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 300, trace=True)
    ga, gb, G = oracle.adjoint(K, prob.a, prob.b, prob.eps, prob.tau, res)
    ea, eb, P = oracle.envelope_gradients(K, res.u, res.v, prob.a, prob.b, prob.tau)
    np.testing.assert_allclose(P, G, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(ea, ga, rtol=0, atol=1e-10)
    np.testing.assert_allclose(eb, gb, rtol=0, atol=1e-10)
    # before convergence they differ: the envelope is not the unrolled gradient
    res5 = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 2, trace=True)
    ga5, _, G5 = oracle.adjoint(K, prob.a, prob.b, prob.eps, prob.tau, res5)
    ea5, _, P5 = oracle.envelope_gradients(K, res5.u, res5.v, prob.a, prob.b, prob.tau)
    assert np.max(np.abs(P5 - G5)) > 1e-6 and np.max(np.abs(ea5 - ga5)) > 1e-6


def test_envelope_gradients_match_finite_differences_of_the_optimum():
    """Central differences of the converged objective in a, b and the cost
    (h = 1e-6 relative), against the envelope gradients."""
    prob = workloads.random_small(6, 5, seed=43, eps=0.4, tau=0.9)
    C, K = _problem_arrays(prob)
    T = 400

    def loss(a, b, C):
        return oracle.sinkhorn(oracle.kernel(C, prob.eps), a, b, prob.eps, prob.tau, T).loss

    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T)
    ea, eb, P = oracle.envelope_gradients(K, res.u, res.v, prob.a, prob.b, prob.tau)
    h = 1e-6
    for i in (0, 3, 5):
        da = np.zeros(6)
        da[i] = h * prob.a[i]
        fd = (loss(prob.a + da, prob.b, C) - loss(prob.a - da, prob.b, C)) / (2 * da[i])
        assert fd == pytest.approx(ea[i], rel=1e-6, abs=1e-9)
    for j in (1, 4):
        db = np.zeros(5)
        db[j] = h * prob.b[j]
        fd = (loss(prob.a, prob.b + db, C) - loss(prob.a, prob.b - db, C)) / (2 * db[j])
        assert fd == pytest.approx(eb[j], rel=1e-6, abs=1e-9)
    for (i, j) in ((0, 0), (2, 3), (5, 4)):
        dC = np.zeros_like(C)
        dC[i, j] = h
        fd = (loss(prob.a, prob.b, C + dC) - loss(prob.a, prob.b, C - dC)) / (2 * h)
        assert fd == pytest.approx(P[i, j], rel=1e-5, abs=1e-11)


# ---------------------------------------------------------------- P10: absorption
def test_stabilized_equals_plain():
    prob = workloads.random_small(14, 10, seed=23, eps=0.02, tau=0.3)
    C, K = _problem_arrays(prob)
    T = 40
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T)
    for thr in (0.0, 0.5, 3.0):
        f, g, nabs = oracle.sinkhorn_stabilized(C, prob.a, prob.b, prob.eps, prob.tau, T, thr)
        np.testing.assert_allclose(f / prob.eps, np.log(res.u), rtol=0, atol=1e-11)
        np.testing.assert_allclose(g / prob.eps, np.log(res.v), rtol=0, atol=1e-11)
        if thr == 0.5:
            assert nabs > 0


def test_absorbed_normalised_equals_plain():
    """The normalised absorbed iteration is a reparameterisation: in FP64 it
    reproduces the plain iterates, marginals and objective for any
    threshold and check interval, also where the plain kernel underflows
    nowhere but exp(-C/eps) spans many decades."""
    prob = workloads.random_small(17, 11, seed=29, eps=0.01, tau=0.2)
    C, K = _problem_arrays(prob)
    T = 60
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T)
    counts = []
    for thr, ce in ((0.0, 1), (0.5, 1), (8.0, 1), (3.0, 7), (1e9, 1)):
        R = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, T, thr, ce)
        np.testing.assert_allclose(R.f / prob.eps, np.log(res.u), rtol=0, atol=1e-10)
        np.testing.assert_allclose(R.g / prob.eps, np.log(res.v), rtol=0, atol=1e-10)
        np.testing.assert_allclose(R.r, res.r, rtol=1e-10)
        np.testing.assert_allclose(R.c, res.c, rtol=1e-10)
        assert R.loss == pytest.approx(res.loss, rel=1e-12)
        counts.append(R.absorptions)
        # a check absorbs exactly when its maximum exceeds the level it is
        # compared against; the level starts at the threshold and never
        # drops below it
        at = R.arms > 0
        assert np.all(R.arms[at] >= thr) and (not np.any(at) or R.arms[at][0] == thr)
        assert int(np.sum(R.checks[at] > R.arms[at])) == R.absorptions
    # 0.5 is below the scale of log a: the first check absorbs, and the
    # residue the normalisation leaves raises the level (no rebuild at every
    # check); 8 absorbs only some of the time
    assert counts[0] == 0 and counts[-1] == 0 and 1 <= counts[1] < T - 1 and counts[2] >= 1
    assert 1 <= counts[3] <= (T - 1) // 7


def test_absorbed_storage_error_scales_with_unit_roundoff():
    """Holding the normalised kernel in binary32 / bfloat16 / E4M3 moves the
    result by an amount that tracks each format's unit roundoff (2^-24,
    2^-8, 2^-4): well below it times the fixed point's amplification and
    ordered like the formats."""
    prob = workloads.random_small(40, 30, seed=31, eps=0.05, tau=0.5)
    C, K = _problem_arrays(prob)
    T = 200
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T)
    fi = prob.tau / (prob.tau + prob.eps)
    amp = fi / (1 - fi)                 # infinity-norm bound of the log fixed point
    errs = {}
    for st, urd, scale in (("f32", 2.0 ** -24, 1.0), ("bf16", 2.0 ** -8, 1.0), ("e4m3", 2.0 ** -4, 448.0)):
        R = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, T, 5.0, 1, st, scale)
        e = max(np.max(np.abs(R.f / prob.eps - np.log(res.u))), np.max(np.abs(R.g / prob.eps - np.log(res.v))))
        errs[st] = e
        assert e <= 2 * amp * urd, (st, e)
    assert errs["f32"] < errs["bf16"] < errs["e4m3"]
    assert errs["bf16"] > 1e-5         # the storage really is applied


# ---------------------------------------------------------------- special cases
def test_zero_mass_entries_and_zero_iterations():
    prob = workloads.random_small(10, 8, seed=24, eps=0.1, tau=0.5)
    C, K = _problem_arrays(prob)
    a = prob.a.copy()
    b = prob.b.copy()
    a[3] = 0.0
    b[5] = 0.0
    res = oracle.sinkhorn(K, a, b, prob.eps, prob.tau, 12)
    assert res.u[3] == 0.0 and res.v[5] == 0.0
    assert res.r[3] == 0.0 and res.c[5] == 0.0
    assert np.all(np.isfinite(res.u)) and np.isfinite(res.loss)
    r0 = oracle.sinkhorn(K, a, b, prob.eps, prob.tau, 0)
    assert r0.iters == 0 and np.all(r0.u == 1.0) and np.all(r0.v == 1.0)
    direct, _ = oracle.loss_direct(C, K, r0.u, r0.v, a, b, prob.eps, prob.tau)
    assert r0.loss == pytest.approx(direct, rel=1e-12)


def test_tolerance_stops_early_and_err_is_relative_l1():
    prob = workloads.random_small(30, 20, seed=25, eps=0.1, tau=0.5)
    C, K = _problem_arrays(prob)
    res = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, 5000, tol=1e-9)
    assert 1 < res.iters < 5000 and res.err <= 1e-9
    r1 = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, res.iters - 1)
    r2 = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, res.iters)
    assert np.sum(np.abs(r2.c - r1.c)) / np.sum(r2.c) == pytest.approx(res.err, rel=1e-9)
    assert np.sum(np.abs(r2.c - r1.c)) / np.sum(r2.c) <= 1e-9
    prev = oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, res.iters - 1, tol=1e-9)
    assert prev.iters == res.iters - 1      # it did not stop earlier


def test_cost_points_kinds():
    rng = np.random.default_rng(3)
    x = rng.random((4, 3))
    y = rng.random((5, 3))
    C = oracle.cost_points(x, y, 0, False)
    assert C[2, 4] == pytest.approx(float(np.sum((x[2] - y[4]) ** 2)), rel=1e-15)
    Cn = oracle.cost_points(x, y, 0, True)
    assert Cn.max() == 1.0
    np.testing.assert_allclose(Cn * C.max(), C, rtol=1e-15)
    Cc = oracle.cost_points(x, y, 1, False)
    assert Cc[1, 3] == pytest.approx(1.0 - float(x[1] @ y[3]), rel=1e-15)


# ---------------------------------------------------------------------------
# Low-precision storage: every representable value and every midpoint
# ---------------------------------------------------------------------------

def _bf16_positive_normals():
    """All positive finite normal bfloat16 values: bit patterns 0x0080..0x7F7F
    placed in the top half of a binary32 word."""
    codes = np.arange(0x0080, 0x7F80, dtype=np.uint32)
    return (codes << 16).view(np.float32).astype(np.float64), codes


def _e4m3_positive_values():
    """All non-negative finite E4M3FN values from the bit layout (bias 7,
    3 fraction bits, subnormals k 2^-9, code 0x7F is NaN)."""
    vals = []
    for code in range(0x00, 0x7F):
        e, k = code >> 3, code & 7
        vals.append(k * 2.0 ** -9 if e == 0 else (1 + k / 8) * 2.0 ** (e - 7))
    return np.array(vals), np.arange(0x00, 0x7F)


def test_round_storage_bf16_grid_and_midpoints():
    vals, codes = _bf16_positive_normals()
    assert np.array_equal(oracle.round_storage(vals, "bf16"), vals)
    lo, hi = vals[:-1], vals[1:]
    mid = (lo + hi) / 2                      # exact in FP64
    even = np.where(codes[:-1] % 2 == 0, lo, hi)
    assert np.array_equal(oracle.round_storage(mid, "bf16"), even)
    assert np.array_equal(oracle.round_storage(np.nextafter(mid, 0), "bf16"), lo)
    assert np.array_equal(oracle.round_storage(np.nextafter(mid, np.inf), "bf16"), hi)
    below = np.array([0.0, 2.0 ** -127, np.nextafter(2.0 ** -126, 0)])
    assert np.all(oracle.round_storage(below, "bf16") == 0.0)


def test_round_storage_bf16_matches_torch_on_binary32_inputs():
    import torch
    rng = np.random.default_rng(11)
    x = np.exp(rng.uniform(-80, 80, 200000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_storage(x.astype(np.float64), "bf16"), ref)


def test_round_storage_e4m3_grid_midpoints_and_saturation():
    vals, codes = _e4m3_positive_values()
    assert vals[-1] == 448.0 and vals[1] == 2.0 ** -9
    assert np.array_equal(oracle.round_storage(vals, "e4m3"), vals)
    lo, hi = vals[:-1], vals[1:]
    mid = (lo + hi) / 2
    even = np.where(codes[:-1] % 2 == 0, lo, hi)
    assert np.array_equal(oracle.round_storage(mid, "e4m3"), even)
    assert np.array_equal(oracle.round_storage(np.nextafter(mid, 0), "e4m3"), lo)
    assert np.array_equal(oracle.round_storage(np.nextafter(mid, np.inf), "e4m3"), hi)
    big = np.array([448.0, 460.0, 464.0, 1e6])
    assert np.all(oracle.round_storage(big, "e4m3") == 448.0)


def test_round_storage_e4m3_matches_torch_in_range():
    import torch
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(0, 448, 100000), np.exp(rng.uniform(-14, 6, 100000))])
    x = x[x <= 448].astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_storage(x.astype(np.float64), "e4m3"), ref)


# ---------------------------------------------------------------------------
# Log-domain (log-sum-exp) iteration and eps-scaling
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eps,tau,zero", [(0.1, 1.0, False), (0.05, math.inf, False), (0.2, 0.5, True)])
def test_lse_equals_vector_form(eps, tau, zero):
    """Same iterates as the vector form on K = exp(-C/eps) (where K is
    representable), zero-mass entries included (u_i = 0 <=> f_i = -inf)."""
    p = workloads.random_small(60, 45, seed=11, eps=eps, tau=tau)
    a, b = p.a.copy(), p.b.copy()
    if zero:
        a[3] = 0.0
        b[7] = 0.0
    C = oracle.cost_points(p.x, p.y)
    ref = oracle.sinkhorn(oracle.kernel(C, eps), a, b, eps, tau, 40)
    lse = oracle.sinkhorn_lse(C, a, b, eps, tau, 40)
    u, v = np.exp(lse.f / eps), np.exp(lse.g / eps)
    assert np.all((u == 0) == (ref.u == 0)) and np.all((v == 0) == (ref.v == 0))
    pos_u, pos_v = ref.u > 0, ref.v > 0
    assert np.max(np.abs(u[pos_u] / ref.u[pos_u] - 1)) < 1e-12
    assert np.max(np.abs(v[pos_v] / ref.v[pos_v] - 1)) < 1e-12
    np.testing.assert_allclose(lse.r, ref.r, rtol=1e-12, atol=0)
    np.testing.assert_allclose(lse.c, ref.c, rtol=1e-12, atol=0)
    assert abs(lse.loss / ref.loss - 1) < 1e-12


def test_lse_one_by_one_closed_form_where_the_kernel_underflows():
    """1 x 1 problem at eps = 1e-4 with C = 3: K = e^-30000 is 0 in FP64, the
    log-domain iterates still follow the closed-form recurrence, and the
    converged plan is the closed-form optimum."""
    a, b, c, eps, tau = 0.7, 1.9, 3.0, 1e-4, 0.5
    for T in (1, 2, 7, 50):
        lu, lv = pins.one_by_one_log(a, b, c, eps, tau, T)
        r = oracle.sinkhorn_lse(np.array([[c]]), np.array([a]), np.array([b]), eps, tau, T)
        assert abs(r.f[0] - eps * lu) <= 1e-13 * max(1.0, abs(eps * lu))
        assert abs(r.g[0] - eps * lv) <= 1e-13 * max(1.0, abs(eps * lv))
    # fi^2 = 0.9996 per iteration: 3e5 iterations leave e^-120 of the start
    r = oracle.sinkhorn_lse(np.array([[c]]), np.array([a]), np.array([b]), eps, tau, 300000)
    P = math.exp((r.f[0] + r.g[0] - c) / eps)
    assert abs(P / pins.one_by_one_limit(a, b, c, eps, tau) - 1) < 1e-10
    # P from potentials carries |C|/eps = 3e4 times the unit roundoff
    assert abs(r.r[0] / P - 1) < 1e-11


@pytest.mark.parametrize("T", [1, 5, 30])
def test_lse_rank1_closed_form_at_small_eps(T):
    """Separable cost alpha_i + beta_j in [0, 2) at eps = 2e-3: kernel entries
    down to e^-1000 (FP64 underflow for the vector form); potentials against
    the closed form of the rank-1 recurrence."""
    rng = np.random.default_rng(21)
    n, m, eps, tau = 70, 50, 2e-3, 0.5
    alpha, beta = rng.random(n), rng.random(m)
    a, b = rng.dirichlet(np.ones(n)), 0.8 * rng.dirichlet(np.ones(m))
    lu, lv = pins.rank1(alpha, beta, a, b, eps, tau, T)
    r = oracle.sinkhorn_lse(np.add.outer(alpha, beta), a, b, eps, tau, T)
    assert np.max(np.abs(r.f - eps * lu)) < 1e-12
    assert np.max(np.abs(r.g - eps * lv)) < 1e-12


def test_lse_tolerance_stop_matches_vector_form():
    p = workloads.random_small(80, 70, seed=12, eps=0.05, tau=1.0)
    C = oracle.cost_points(p.x, p.y)
    ref = oracle.sinkhorn(oracle.kernel(C, p.eps), p.a, p.b, p.eps, p.tau, 5000, tol=1e-9)
    lse = oracle.sinkhorn_lse(C, p.a, p.b, p.eps, p.tau, 5000, tol=1e-9)
    assert 10 < ref.iters < 5000 and lse.iters == ref.iters
    # the error is a difference of nearly equal marginals: compare absolutely
    assert abs(lse.err - ref.err) < 1e-14


def test_eps_scaling_schedule_and_fixed_point():
    """Stages at eps0 factor^k down to eps (each stage_iters iterations, the
    last up to max_iter): a fixed count runs sum of stages; a schedule that
    starts at eps is the plain run; a converged scaled run reaches the plain
    run's fixed point (unique for tau < inf)."""
    p = workloads.random_small(40, 30, seed=13, eps=0.01, tau=1.0)
    C = oracle.cost_points(p.x, p.y)
    # stages 0.16, 0.08, 0.04, 0.02 (3 iterations each), then 0.01 (5)
    r = oracle.sinkhorn_lse(C, p.a, p.b, 0.01, 1.0, 5, eps0=0.16, factor=0.5, stage_iters=3)
    assert r.iters == 4 * 3 + 5
    plain = oracle.sinkhorn_lse(C, p.a, p.b, 0.01, 1.0, 7)
    same = oracle.sinkhorn_lse(C, p.a, p.b, 0.01, 1.0, 7, eps0=0.01, factor=0.5, stage_iters=9)
    assert np.array_equal(plain.f, same.f) and np.array_equal(plain.g, same.g)
    direct = oracle.sinkhorn_lse(C, p.a, p.b, 0.01, 1.0, 100000, tol=1e-14)
    scaled = oracle.sinkhorn_lse(C, p.a, p.b, 0.01, 1.0, 100000, tol=1e-14, eps0=1.0, factor=0.5, stage_iters=20)
    assert direct.iters < 100000 and scaled.iters < 100000
    assert np.max(np.abs(scaled.f - direct.f)) < 1e-9 and np.max(np.abs(scaled.g - direct.g)) < 1e-9
