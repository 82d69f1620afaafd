"""Low-precision K storage (FP32, BF16, FP8-E4M3) with log-domain absorption.

Each storage type is checked two ways:
  parity         against the oracle running the same iteration on the same
                 stored kernel values (the oracle rounds with its own code,
                 written from the format definitions): what is left is the
                 GPU's arithmetic (FP32 products and lane sums, FP64
                 reductions), held to the FP32 tolerance;
  storage error  against the plain FP64 oracle (exact kernel), reported for
                 u, v and the loss.  BF16 is held to 2e-3 as a normwise
                 relative error.  Entry by entry no bfloat16-stored kernel can
                 meet it: one rounding moves an entry by up to 2^-8, and the
                 oracle's own exact-arithmetic BF16 run moves single u_i by
                 ~3.7e-3 here.  FP8 has no bar.

Errors of u, v are computed from the potentials f = eps log u so that they
stay meaningful where u itself overflows: entrywise |expm1((f - f_ref)/eps)|;
normwise ||U - U_ref||_2 / ||U_ref||_2 with U = exp((f - max f_ref)/eps)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu

import paper_2412_11079_amd as uot  # noqa: E402

STORE = {torch.float64: (None, 1.0), torch.float32: ("f32", 1.0), torch.bfloat16: ("bf16", 1.0),
         torch.float8_e4m3fn: ("e4m3", uot.FP8_STORE_SCALE)}
UNIT_ROUNDOFF = {torch.float32: 2.0 ** -24, torch.bfloat16: 2.0 ** -8, torch.float8_e4m3fn: 2.0 ** -4}


def e4m3fn_decode(byte: int) -> float:
    """OCP E4M3FN: sign, 4 exponent bits (bias 7), 3 mantissa bits; 0x7F and
    0xFF are NaN; no infinities."""
    s = -1.0 if byte & 0x80 else 1.0
    e = (byte >> 3) & 0xF
    mnt = byte & 7
    if e == 15 and mnt == 7:
        return math.nan
    if e == 0:
        return s * mnt * 2.0 ** -9
    return s * (1.0 + mnt / 8.0) * 2.0 ** (e - 7)


def test_fp8_decode_is_ocp_e4m3fn():
    codes = torch.arange(256, dtype=torch.uint8, device="cuda").view(torch.float8_e4m3fn)
    got = uot.kernel_to_f32(codes).cpu().numpy().astype(np.float64)
    ref = np.array([e4m3fn_decode(b) for b in range(256)])
    nan = np.isnan(ref)
    assert np.all(np.isnan(got[nan]))
    np.testing.assert_array_equal(got[~nan], ref[~nan])


def _normalised_potentials(C):
    f = C.min(axis=1)
    g = (C - f[:, None]).min(axis=0)
    return f, g


def _oracle_stored_kernel(C, eps, f, g, dtype):
    kind, scale = STORE[dtype]
    K = oracle.kernel(C, eps, f, g)
    if kind is None:
        return K
    return oracle.round_storage(K * scale, kind) / scale


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float8_e4m3fn])
def test_kernel_build_rounding_matches_oracle_storage(dtype):
    """Stored kernel entries equal the oracle's rounding of the same FP64
    values, bit for bit (FP8 holds 448 K; decoded and divided back here)."""
    prob = workloads.precision(n=70, m=300, max_iter=1)
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    f, g = _normalised_potentials(C)
    Kd = uot.kernel_from_cost(to_dev(C), prob.eps, dtype, f=to_dev(f), g=to_dev(g))
    scale = STORE[dtype][1]
    got = uot.kernel_to_f32(Kd).cpu().numpy().astype(np.float64)[:, :300] / scale
    ref = _oracle_stored_kernel(C, prob.eps, f, g, dtype)
    assert np.array_equal(got, ref)
    assert np.all(uot.kernel_to_f32(Kd).cpu().numpy()[:, 300:] == 0)      # padding columns
    assert got.max() == 1.0


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


@pytest.mark.parametrize("m", [1111, 7999])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float8_e4m3fn])
def test_stored_kernel_iteration_matches_oracle_on_same_kernel(dtype, m):
    """Without absorption (eps = 0.02, so the normalised kernel spans e^-50
    .. 1): a stored K given to uot_sinkhorn against the oracle's plain
    iteration on the oracle's rounding of the same K.  Ragged n, m; m = 7999
    takes the 512-lane row-batched launch shapes of each storage type."""
    prob = workloads.precision(n=3001 if m < 4000 else 1001, m=m, max_iter=120)
    prob.eps = 0.02
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    f, g = _normalised_potentials(C)
    Kr = _oracle_stored_kernel(C, prob.eps, f, g, dtype)
    ref = oracle.sinkhorn(Kr, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter)
    Kd = uot.kernel_from_cost(to_dev(C), prob.eps, dtype, f=to_dev(f), g=to_dev(g))
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), Kd, m=prob.m, eps=prob.eps, tau=prob.tau,
                       max_iter=prob.max_iter)
    torch.cuda.synchronize()
    info = res.info()
    eu = _rel(res.u.cpu().numpy(), ref.u)
    ev = _rel(res.v.cpu().numpy(), ref.v)
    el = abs(float(res.loss.cpu()) - ref.loss) / abs(ref.loss)
    say(f"  {dtype}: u {eu:.3e} v {ev:.3e} loss {el:.3e}")
    assert info["flags"] == 0 and info["iters"] == prob.max_iter
    assert eu <= 1e-6 and ev <= 1e-6 and el <= 1e-6


def _gpu_absorbed(prob, dtype, check_every=1, thr=30.0, C=None):
    if C is None:
        C = uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), prob.cost_kind, prob.normalize_max)
    res = uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), None, C=C, k_dtype=dtype, eps=prob.eps, tau=prob.tau,
                       max_iter=prob.max_iter, absorb_log_threshold=thr, check_every=check_every)
    torch.cuda.synchronize()
    return res


def _decision_margin(res) -> float:
    """Smallest |max |log| - level| over the oracle's absorption checks."""
    at = res.arms > 0
    return float(np.min(np.abs(res.checks[at] - res.arms[at]))) if np.any(at) else math.inf


def _pot_errors(f, g, f0, g0, eps):
    """(entrywise max u, entrywise max v, normwise u, normwise v)."""
    du = np.expm1((f - f0) / eps)
    dv = np.expm1((g - g0) / eps)
    wu = np.exp((f0 - f0.max()) / eps)
    wv = np.exp((g0 - g0.max()) / eps)
    nu = float(np.linalg.norm(du * wu) / np.linalg.norm(wu))
    nv = float(np.linalg.norm(dv * wv) / np.linalg.norm(wv))
    return float(np.max(np.abs(du))), float(np.max(np.abs(dv))), nu, nv


# Parity bars of the absorbed iteration at eps = 1e-3 (fi = 0.990): FP32
# arithmetic is amplified by the fixed point, ~1/(1 - fi^2) = 50.
ABSORBED_PARITY = {torch.float64: 1e-10, torch.float32: 2e-5, torch.bfloat16: 2e-5, torch.float8_e4m3fn: 2e-5}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float8_e4m3fn])
def test_absorbed_iteration_against_oracle(dtype):
    """Precision workload shape (16-D normal points, eps 1e-3, tau 0.1,
    threshold 30) at 4096 x 1024, 300 iterations."""
    prob = workloads.precision(n=4096, m=1024, max_iter=300)
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    kind, scale = STORE[dtype]
    same = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, 30.0, 1, kind, scale)
    # the schedule is decided far enough from the compared level for FP32 sums
    assert _decision_margin(same) > 1e-3
    res = _gpu_absorbed(prob, dtype)
    info = res.info()
    f, g = res.f.cpu().numpy(), res.g.cpu().numpy()
    eu, ev, nu, nv = _pot_errors(f, g, same.f, same.g, prob.eps)
    el = abs(float(res.loss.cpu()) - same.loss) / abs(same.loss)
    say(f"  {dtype} vs oracle on the same storage: u {eu:.3e} v {ev:.3e} loss {el:.3e}; "
        f"absorptions {info['absorptions']} (oracle {same.absorptions})")
    assert info["iters"] == 300 and info["flags"] == 0
    assert info["absorptions"] == same.absorptions >= 1
    bar = ABSORBED_PARITY[dtype]
    assert eu <= bar and ev <= bar and el <= bar
    np.testing.assert_allclose(res.r.cpu().numpy(), same.r, rtol=bar, atol=0)
    np.testing.assert_allclose(res.c.cpu().numpy(), same.c, rtol=bar, atol=0)

    # storage error: against the exact FP64 kernel
    ref, _, _ = oracle.solve_problem(prob)
    f0, g0 = prob.eps * np.log(ref.u), prob.eps * np.log(ref.v)
    eu, ev, nu, nv = _pot_errors(f, g, f0, g0, prob.eps)
    el = abs(float(res.loss.cpu()) - ref.loss) / abs(ref.loss)
    say(f"  {dtype} vs FP64 oracle: entrywise u {eu:.3e} v {ev:.3e}; normwise u {nu:.3e} v {nv:.3e}; "
        f"loss {el:.3e}")
    if dtype == torch.float64:
        assert max(eu, ev, el) <= 1e-10
    elif dtype == torch.float32:
        assert max(eu, ev, el) <= 2e-5
    elif dtype == torch.bfloat16:
        assert max(nu, nv, el) <= 2e-3


def test_absorption_schedule_does_not_change_fp64_result():
    prob = workloads.precision(n=1024, m=512, max_iter=120)
    ref, _, _ = oracle.solve_problem(prob)
    f0, g0 = prob.eps * np.log(ref.u), prob.eps * np.log(ref.v)
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    counts = []
    for ce, thr in ((1, 30.0), (7, 30.0), (1, 5.0), (3, 1e9)):
        res = _gpu_absorbed(prob, torch.float64, check_every=ce, thr=thr)
        eu, ev, _, _ = _pot_errors(res.f.cpu().numpy(), res.g.cpu().numpy(), f0, g0, prob.eps)
        el = abs(float(res.loss.cpu()) - ref.loss) / abs(ref.loss)
        counts.append(res.info()["absorptions"])
        same = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, thr, ce)
        say(f"  check_every={ce} thr={thr}: {eu:.2e} {ev:.2e} {el:.2e} abs={counts[-1]} "
            f"(oracle {same.absorptions}, margin {_decision_margin(same):.2e})")
        assert eu <= 1e-10 and ev <= 1e-10 and el <= 1e-10
        if _decision_margin(same) > 1e-6:
            assert counts[-1] == same.absorptions
    assert counts[3] == 0 and counts[0] >= 1 and counts[2] > counts[0]


@pytest.mark.parametrize("m", [3000, 8192, 9000])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float8_e4m3fn])
def test_absorbed_rebuild_paths_same_storage(dtype, m):
    """The normalised kernel build at the column counts of each rebuild
    kernel: row and column minima in one read of C with 4 (m = 3000) or 8
    (m = 8192, the precision workload's width) columns per lane, and
    separate row and column minima (m = 9000); then 6 iterations of the
    absorbed passes on it (no absorption yet: the level is out of reach, so
    the stored kernel comes from C alone and matches the oracle's bit for
    bit).  Against the oracle on the same storage at each form's parity bar."""
    if dtype == torch.float64 and m > 8192:
        pytest.skip("FP64 rows hold at most 8192 columns")
    prob = workloads.precision(n=1000, m=m, max_iter=6)
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    kind, scale = STORE[dtype]
    same = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, 1e9, 1, kind, scale)
    res = _gpu_absorbed(prob, dtype, check_every=1, thr=1e9)
    info = res.info()
    f, g = res.f.cpu().numpy(), res.g.cpu().numpy()
    eu, ev, _, _ = _pot_errors(f, g, same.f, same.g, prob.eps)
    el = abs(float(res.loss.cpu()) - same.loss) / abs(same.loss)
    say(f"rebuild path {dtype} n=1000 m={m}: u {eu:.3e} v {ev:.3e} loss {el:.3e} (largest |log| "
        f"{same.checks.max():.1f})")
    assert info["iters"] == 6 and info["flags"] == 0 and info["absorptions"] == 0
    bar = ABSORBED_PARITY[dtype]
    assert eu <= bar and ev <= bar and el <= bar
    np.testing.assert_allclose(res.r.cpu().numpy(), same.r, rtol=bar, atol=0)
    np.testing.assert_allclose(res.c.cpu().numpy(), same.c, rtol=bar, atol=0)


@pytest.mark.parametrize("m", [3000, 8192, 9000])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float8_e4m3fn])
def test_absorbed_iteration_with_rebuilds(dtype, m):
    """200 iterations with absorption (level 30, checked every iteration)
    at the three rebuild paths' column counts.  FP64 and FP32: against the
    oracle on the same storage and schedule (same absorption count) and
    against the plain FP64 iteration.  BF16, FP8: after an absorption the
    potentials carry the GPU's FP32 rounding, so a few stored entries may
    round to the neighbouring code and the same-storage comparison is only
    as tight as one storage rounding; held instead to the storage bar against
    the plain FP64 iteration (BF16: 2e-3 normwise on u, v and the loss; FP8:
    finite, reported)."""
    if dtype == torch.float64 and m > 8192:
        pytest.skip("FP64 rows hold at most 8192 columns")
    prob = workloads.precision(n=1000, m=m, max_iter=200)
    C = oracle.cost_points(prob.x, prob.y, 0, True)
    kind, scale = STORE[dtype]
    same = oracle.sinkhorn_absorbed(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, 30.0, 1, kind, scale)
    res = _gpu_absorbed(prob, dtype, check_every=1)
    info = res.info()
    f, g = res.f.cpu().numpy(), res.g.cpu().numpy()
    assert info["iters"] == 200 and info["flags"] == 0 and info["absorptions"] >= 1
    if _decision_margin(same) > 1e-3:
        assert info["absorptions"] == same.absorptions
    # the plain FP64 iteration (textbook stabilised form, its own absorption rule)
    f0, g0, _ = oracle.sinkhorn_stabilized(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, 30.0)
    r0, c0 = oracle.potential_marginals(C, f0, g0, prob.eps)
    L0 = oracle.loss_potentials(f0, g0, r0, c0, prob.a, prob.b, prob.eps, prob.tau)
    eu, ev, nu, nv = _pot_errors(f, g, f0, g0, prob.eps)
    el = abs(float(res.loss.cpu()) - L0) / abs(L0)
    say(f"absorbed {dtype} n=1000 m={m}: absorptions {info['absorptions']} (oracle {same.absorptions}); vs plain "
        f"FP64: entrywise u {eu:.3e} v {ev:.3e}, normwise u {nu:.3e} v {nv:.3e}, loss {el:.3e}")
    if dtype in (torch.float64, torch.float32):
        bar = ABSORBED_PARITY[dtype]
        su, sv, _, _ = _pot_errors(f, g, same.f, same.g, prob.eps)
        sl = abs(float(res.loss.cpu()) - same.loss) / abs(same.loss)
        assert su <= bar and sv <= bar and sl <= bar
        tol = 1e-10 if dtype == torch.float64 else 2e-5
        assert eu <= tol and ev <= tol and el <= tol
    elif dtype == torch.bfloat16:
        assert max(nu, nv, el) <= 2e-3
    else:
        assert np.all(np.isfinite(f)) and np.all(np.isfinite(g)) and math.isfinite(el)


def test_absorption_needs_cost():
    prob = workloads.precision(n=64, m=64, max_iter=3)
    C = uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), 0, True)
    K = uot.kernel_from_cost(C, prob.eps, torch.float32)
    with pytest.raises(uot.UOTError) as e:
        uot.sinkhorn(to_dev(prob.a), to_dev(prob.b), K, eps=prob.eps, tau=prob.tau, max_iter=3,
                     absorb_log_threshold=30.0)
    assert e.value.status == 1


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision_65536x8192_fp64.npz")


def precision_reference():
    """FP64 oracle result of the precision workload at full size, written by
    tests/golden/make_precision_reference.py (oracle only)."""
    z = np.load(GOLDEN)
    return {k: z[k] for k in z.files}


def test_precision_full_size():
    """65536 x 8192, eps 1e-3, threshold 30, 2000 iterations, checks every
    10, K stored in FP32, BF16 and FP8, against the FP64 oracle's result at
    the same size (stabilised FP64 iteration, stored under tests/golden).
    Bars: FP32 1e-6 on the loss and, on u and v entry by entry, the stored
    kernel's own bound 2 fi/(1 - fi) 2^-24 = 1.2e-5 (one rounding of each
    entry, amplified by the fixed point at fi = 0.990); BF16 2e-3 normwise
    on u, v and on the loss (entrywise reported); FP8 reported.  FP8 checks
    the scalings every 2 iterations (its truncated kernel moves them by up to
    ~7 log units per iteration, and the passes' FP32 lane products hold
    |log| < 88); it must not absorb far more often than FP32 (a rebuild that
    the normalisation undoes is not repeated)."""
    ref = precision_reference()
    prob = workloads.precision()
    assert int(ref["n"]) == prob.n and int(ref["m"]) == prob.m and int(ref["iters"]) == prob.max_iter
    Cd = uot.cost_from_points(to_dev(prob.x), to_dev(prob.y), prob.cost_kind, prob.normalize_max)
    counts = {}
    for dtype in (torch.float32, torch.bfloat16, torch.float8_e4m3fn):
        say(f"  full size {dtype} ...")
        r = _gpu_absorbed(prob, dtype, check_every=2 if dtype == torch.float8_e4m3fn else 10, C=Cd)
        info = r.info()
        counts[dtype] = info["absorptions"]
        eu, ev, nu, nv = _pot_errors(r.f.cpu().numpy(), r.g.cpu().numpy(), ref["f"], ref["g"], prob.eps)
        el = abs(float(r.loss.cpu()) - float(ref["loss"])) / abs(float(ref["loss"]))
        say(f"    vs FP64 oracle: entrywise u {eu:.3e} v {ev:.3e}; normwise u {nu:.3e} v {nv:.3e}; "
            f"loss {el:.3e}; absorptions {info['absorptions']} flags {info['flags']}")
        assert info["flags"] == 0 and info["iters"] == 2000 and info["absorptions"] >= 1
        if dtype == torch.float32:
            fi = prob.tau / (prob.tau + prob.eps)
            assert max(eu, ev) <= 2 * fi / (1 - fi) * 2.0 ** -24 and el <= 1e-6
        elif dtype == torch.bfloat16:
            assert max(nu, nv, el) <= 2e-3
        else:
            assert np.isfinite(eu) and np.isfinite(ev) and np.isfinite(el)
    assert counts[torch.float8_e4m3fn] <= 5 * counts[torch.float32] + 5
