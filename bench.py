"""Benchmark of the UOT Sinkhorn hot path on one MI355X.

One step = the whole path on the headline workload: FP64 cost from the
3-D point clouds, Gibbs kernel build (FP32), 1000 fused single-pass
iterations (row and column half-steps), final marginals and FP64
objective.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line (rank 0).  Besides the contract fields it carries:
  roofline      the fused pass kernel: algorithmic bytes (N*M*4 per launch)
                over its average launch duration (HIP events recorded by
                the library on the launch stream during the timed steps);
  cpu_baseline  the FP64 oracle on the host cores, bounded sample;
  plain         the plain two-pass form on the same GPU (same steps);
  fwd_bwd       forward + reverse pass of the differentiation workload;
  batched       1024 uneven problems in one persistent launch;
  multi         256 histogram pairs sharing one 8192^2 kernel (matrix cores);
  precision     65536 x 8192 with BF16 / FP8 / FP32 K and absorption;
  kernel_free   the kernel-free solve (K recomputed in every pass) on the
                3-D differentiation and 2-D plain workloads, against the
                streamed FP32 K at the same shapes, with its ALU roofline;
  log_domain    the log-domain (log-sum-exp) solve on the precision workload
                (FP64 and FP32 cost, no absorption) with its errors against
                the FP64 oracle, and eps-scaling against the direct run to a
                tolerance.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Sinkhorn iters/s + achieved HBM TB/s at N=M=16384 FP32; fwd+bwd ms"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_pass_headline_traffic.txt")
# sources of the fused pass kernel: counter results are tied to their hash
PASS_SRC = [os.path.join(ROOT, "paper_2412_11079_amd", "csrc", f) for f in ("pass.hip", "strip.h", "uot_common.h")]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--iters", type=int, default=1000, help="iterations per step")
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--m", type=int, default=16384)
    p.add_argument("--tune", type=int, default=0)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    p.add_argument("--no-plain", action="store_true", help="skip the plain two-pass comparison")
    p.add_argument("--no-grad", action="store_true", help="skip the forward+backward timing")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-problems timing")
    p.add_argument("--no-multi", action="store_true", help="skip the multi-right-hand-side timing")
    p.add_argument("--no-precision", action="store_true", help="skip the low-precision timing")
    p.add_argument("--no-kernel-free", action="store_true", help="skip the kernel-free solve timing")
    p.add_argument("--no-log-domain", action="store_true", help="skip the log-domain solve timing")
    p.add_argument("--only", default="", help="comma list of sections to run alone (profiling)")
    p.add_argument("--cpu-leg", type=int, default=0, help=argparse.SUPPRESS)
    p.add_argument("--cpu-rows", type=int, default=0, help=argparse.SUPPRESS)
    p.add_argument("--cpu-reps", type=int, default=1, help=argparse.SUPPRESS)
    p.add_argument("--calib-copy", action="store_true",
                   help="only run a plain device copy of known size (counter calibration)")
    return p.parse_args()


def src_hash() -> str:
    h = hashlib.sha256()
    for path in PASS_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters():
    """HBM bytes per fused launch from committed rocprofv3 counter runs, or
    None when absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                t[k] = v
    if t.get("pass_src_sha256_16") != src_hash():
        return None
    return int(t["bytes_per_launch"])


def main():
    args = parse()
    if args.cpu_leg > 0:
        cpu_leg(args.cpu_leg, args.cpu_rows, args.cpu_reps)
        return
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU (--gpus 1): this path runs on a single MI355X; "
                 "a run over several GPUs is not built")
    import numpy as np
    import torch

    import paper_2412_11079_amd as uot
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)

    if args.only:
        sections = {"grad": fwd_bwd, "batched": batched, "multi": multi, "precision": precision,
                    "kernel_free": kernel_free, "log_domain": log_domain}
        res = {k: sections[k](uot, workloads, torch, dev, args) for k in args.only.split(",")}
        print(json.dumps(res), flush=True)
        return

    if args.calib_copy:
        nbytes = 1 << 30
        x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes, "launches": 5}), flush=True)
        return

    prob = workloads.headline(n=args.n, m=args.m, max_iter=args.iters)
    x = torch.from_numpy(prob.x).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    a = torch.from_numpy(prob.a).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    torch.cuda.synchronize()

    def step(fused: bool, profile: bool):
        C = uot.cost_from_points(x, y, prob.cost_kind, prob.normalize_max)
        K = uot.kernel_from_cost(C, prob.eps, torch.float32)
        del C
        return uot.sinkhorn(a, b, K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=args.iters, tol=0.0,
                            fused=fused, tune=args.tune, profile=profile)

    def run(fused: bool):
        for _ in range(args.warmup):
            step(fused, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pass_ms = 0.0
        launches = 0
        fin_ms = 0.0
        last = None
        for _ in range(args.steps):
            last = step(fused, True)
            p = last.profile
            if fused:
                pass_ms += p["fused_ms"]
                launches += p["fused_launches"]
            else:
                pass_ms += p["row_ms"] + p["col_ms"]
                launches += p["row_launches"] + p["col_launches"]
            fin_ms += p["finalize_ms"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = last.info()
        assert info["iters"] == args.iters and info["flags"] == 0, info
        ms_step = (t1 - t0) * 1e3 / args.steps
        return {"ms_per_step": ms_step, "iters_per_s": args.iters * 1e3 / ms_step,
                "pass_us": pass_ms * 1e3 / max(launches, 1), "finalize_us": fin_ms * 1e3 / max(launches, 1),
                "loss": float(last.loss.cpu())}

    fused = run(True)
    nbytes = prob.n * prob.m * 4
    achieved = nbytes / (fused["pass_us"] * 1e-6) / 1e9
    out = {
        "metric": METRIC,
        "value": round(fused["iters_per_s"], 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fused["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"headline UOT Sinkhorn: fused single pass, FP32 K, N={prob.n} M={prob.m}, "
                               "3-D 8-component GMM points (sigma 0.1), sq-Euclidean cost / max, "
                               f"a,b Dirichlet(1), b mass 0.8, eps={prob.eps}, tau={prob.tau}, "
                               f"{args.iters} iterations per step (cost + kernel build + loop + objective)",
                   "n": prob.n, "m": prob.m, "iters_per_step": args.iters, "parallelism": "single GPU"},
        "hbm_tb_s": round(achieved / 1e3, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_counters(),
                     "kernel": "pass_kernel<float,float,...,MODE_FUSED>",
                     "bytes_per_launch": nbytes, "avg_launch_us": round(fused["pass_us"], 2)},
        "finalize_us": round(fused["finalize_us"], 2),
    }
    if not args.no_plain:
        plain = run(False)
        out["plain"] = {"iters_per_s": round(plain["iters_per_s"], 2), "ms_per_step": round(plain["ms_per_step"], 3),
                        "pass_us": round(plain["pass_us"], 2),
                        "hbm_tb_s": round(nbytes / (plain["pass_us"] * 1e-6) / 1e12, 3),
                        "speedup_fused_over_plain": round(fused["iters_per_s"] / plain["iters_per_s"], 3)}
    if not args.no_plain:
        out["paper_literal"] = paper_literal(uot, workloads, torch, dev, args, prob, fused["iters_per_s"])
    if not args.no_grad:
        out["fwd_bwd"] = fwd_bwd(uot, workloads, torch, dev, args)
    if not args.no_batched:
        out["batched"] = batched(uot, workloads, torch, dev, args)
    if not args.no_multi:
        out["multi"] = multi(uot, workloads, torch, dev, args)
    if not args.no_precision:
        out["precision"] = precision(uot, workloads, torch, dev, args)
    if not args.no_kernel_free:
        out["kernel_free"] = kernel_free(uot, workloads, torch, dev, args)
    if not args.no_log_domain:
        out["log_domain"] = log_domain(uot, workloads, torch, dev, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


def paper_literal(uot, workloads, torch, dev, args, prob, fused_its):
    """The paper's literal in-place form on the headline matrix (16384^2
    FP32): each iteration reads and writes the matrix once (fused), so twice
    the bytes of the vector form's single read.  Timed on the same number of
    iterations per step."""
    C = uot.cost_from_points(torch.from_numpy(prob.x).to(dev), torch.from_numpy(prob.y).to(dev),
                             prob.cost_kind, prob.normalize_max)
    K = uot.kernel_from_cost(C, prob.eps, torch.float32)
    del C
    a = torch.from_numpy(prob.a).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    A = K.clone()
    uot.matrix_rescale_(A, a, b, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=5)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    A.copy_(K)
    e0.record()
    r = uot.matrix_rescale_(A, a, b, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=args.iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert r.info()["flags"] == 0
    its = args.iters / (ms * 1e-3)
    return {"workload": f"paper-literal in-place rescaling of the {prob.n}x{prob.m} FP32 headline matrix, "
                        f"{args.iters} iterations (read + write of A per iteration)",
            "iters_per_s": round(its, 2), "ms_per_solve": round(ms, 3),
            "hbm_tb_s": round(2 * prob.n * prob.m * 4 * its / 1e12, 3),
            "speedup_vector_fused_over_literal": round(fused_its / its, 3)}


def fwd_bwd(uot, workloads, torch, dev, args):
    """Differentiation workload (8192^2 FP32 K, 500 iterations, checkpoints
    every 50): forward (cost, kernel, loop, objective) and reverse pass with
    gradients for the source points, a and b, timed with events on the stream."""
    prob = workloads.grad()
    x = torch.from_numpy(prob.x).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    a = torch.from_numpy(prob.a).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    g = torch.ones((), dtype=torch.float64, device=dev)

    def fwd():
        C = uot.cost_from_points(x, y)
        K = uot.kernel_from_cost(C, prob.eps, torch.float32)
        del C
        return uot.sinkhorn(a, b, K, eps=prob.eps, tau=prob.tau, max_iter=prob.max_iter,
                            checkpoint_every=prob.checkpoint_every)

    for _ in range(max(args.warmup, 1)):
        r = fwd()
        uot.sinkhorn_backward(r, g, x=x, y=y)
    torch.cuda.synchronize()
    reps = max(min(args.steps, 5), 1)
    f_ms = b_ms = 0.0
    for _ in range(reps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        r = fwd()
        e1.record()
        uot.sinkhorn_backward(r, g, x=x, y=y)
        e2.record()
        torch.cuda.synchronize()
        f_ms += e0.elapsed_time(e1)
        b_ms += e1.elapsed_time(e2)
    f_ms /= reps
    b_ms /= reps
    # the same reverse pass also forming the dense dL/dC and dL/dy
    c_ms = 0.0
    for _ in range(reps):
        r = fwd()
        e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e1.record()
        gr = uot.sinkhorn_backward(r, g, x=x, y=y, want_C=True, want_y=True)
        e2.record()
        torch.cuda.synchronize()
        c_ms += e1.elapsed_time(e2)
        del gr
    c_ms /= reps
    # every iterate stored by the forward (131 MB at 8192^2, T = 500): the
    # reverse pass repeats no forward pass
    s_fms = s_bms = 0.0
    for _ in range(reps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        C = uot.cost_from_points(x, y)
        K = uot.kernel_from_cost(C, prob.eps, torch.float32)
        del C
        rs = uot.sinkhorn(a, b, K, eps=prob.eps, tau=prob.tau, max_iter=prob.max_iter, store_iterates=True)
        e1.record()
        gs = uot.sinkhorn_backward(rs, g, x=x, y=y)
        e2.record()
        torch.cuda.synchronize()
        if _ > 0:       # the first round allocates the record
            s_fms += e0.elapsed_time(e1)
            s_bms += e1.elapsed_time(e2)
    s_fms /= reps
    s_bms /= reps
    gc = uot.sinkhorn_backward(fwd(), g, x=x, y=y)
    torch.cuda.synchronize()
    stored_same = all(torch.equal(getattr(gs, k), getattr(gc, k)) for k in ("grad_a", "grad_b", "grad_x"))
    del rs, gs, gc, K
    # implicit (envelope) gradients at the final scalings: no checkpoints
    r = uot.sinkhorn(a, b, uot.kernel_from_cost(uot.cost_from_points(x, y), prob.eps, torch.float32), eps=prob.eps,
                     tau=prob.tau, max_iter=prob.max_iter)
    i_ms = 0.0
    for _ in range(reps + 1):
        e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e1.record()
        gi = uot.sinkhorn_implicit_backward(r, g, x=x, y=y, want_C=False, want_y=True)
        e2.record()
        torch.cuda.synchronize()
        i_ms = e1.elapsed_time(e2) if i_ms == 0.0 else min(i_ms, e1.elapsed_time(e2))
    gu = uot.sinkhorn_backward(fwd(), g, x=x, y=y)
    torch.cuda.synchronize()
    imp_err = {k: float(f"{(torch.linalg.norm(getattr(gi, k) - getattr(gu, k)) / torch.linalg.norm(getattr(gu, k))).item():.3e}")
               for k in ("grad_a", "grad_b", "grad_x")}
    kb = prob.n * prob.m * 4
    # forward: T passes; reverse: T recompute + T adjoint passes + 1 column + 1 seed pass
    passes = prob.max_iter * 3 + 3
    return {"workload": f"grad: N=M={prob.n} FP32 K, {prob.max_iter} iterations, checkpoints every "
                        f"{prob.checkpoint_every}, gradients for x, a, b",
            "fwd_ms": round(f_ms, 3), "bwd_ms": round(b_ms, 3), "fwd_bwd_ms": round(f_ms + b_ms, 3),
            "bwd_with_cost_grad_ms": round(c_ms, 3),
            "stored_iterates": {"fwd_ms": round(s_fms, 3), "bwd_ms": round(s_bms, 3),
                                "fwd_bwd_ms": round(s_fms + s_bms, 3), "grads_equal_checkpointed": stored_same},
            "implicit_bwd_ms": round(i_ms, 3), "implicit_vs_unrolled_normwise": imp_err,
            "cost_grad_tflop_s": round(2.0 * prob.n * prob.m * (2 * prob.max_iter + 2) / ((c_ms - b_ms) * 1e-3) / 1e12, 2)
            if c_ms > b_ms else None,
            "k_passes": passes, "k_bytes_tb_s": round(passes * kb / ((f_ms + b_ms) * 1e-3) / 1e12, 3)}


# VALU issue slots per entry of the kernel-free pass (FP64 exponent: one
# add and one FMA per coordinate, rint, subtract, FP32 conversion, clamp and
# integer conversion; exp2, which issues at half rate, counts two; ldexp;
# the row-dot and column FMAs), and the chip's lane-slot rate:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
KF_SLOTS_PER_ENTRY = {2: 13, 3: 14}
# Rows wider than 8192 columns (column tiles): every entry is formed twice,
# in the row pass (exponent, exp2, ldexp, one FMA with v) and in the column
# pass (the same with u): 12 or 13 slots each.
KF_TILED_SLOTS_PER_ENTRY = {2: 24, 3: 26}
LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


def kernel_free(uot, workloads, torch, dev, args):
    """Kernel-free solve (K recomputed from the points in every pass) on the
    differentiation workload's forward problem (8192^2, 3-D, eps 0.02, 500
    iterations), the plain 2-D workload (1024^2, eps 0.05, 100 iterations)
    and the headline workload (16384^2 3-D mixture, max-normalised cost,
    200 iterations: column tiles, a row pass and a column pass per
    iteration), against the streamed FP32 K on the same problems (cost and
    kernel build included, as the kernel-free solve includes its setup).
    Per-iteration time from two solves of T and 2T iterations (setup
    cancels); it covers the pass and the column finalize, so the ALU
    fraction is a lower bound."""
    import numpy as np
    out = {}
    for key, prob, T in (("diff_8192x8192_3d", workloads.grad(), 500), ("plain_1024x1024_2d", workloads.plain_fp64(), 100),
                         ("headline_16384x16384_3d_tiles", workloads.headline(), 200)):
        x = torch.from_numpy(prob.x).to(dev)
        y = torch.from_numpy(prob.y).to(dev)
        a = torch.from_numpy(prob.a).to(dev)
        b = torch.from_numpy(prob.b).to(dev)
        d = prob.x.shape[1]
        scale = 1.0
        if prob.normalize_max:         # the max-normalised cost as a scale of the plain one
            C0 = uot.cost_from_points(x, y, prob.cost_kind, False)
            scale = 1.0 / float(C0.max())
            del C0
        tiled = prob.m > 8192
        slots = (KF_TILED_SLOTS_PER_ENTRY if tiled else KF_SLOTS_PER_ENTRY)[d]

        def online(T_):
            return uot.sinkhorn_points(x, y, a, b, eps=prob.eps, tau=prob.tau, max_iter=T_, cost_scale=scale)

        def streamed(T_):
            C = uot.cost_from_points(x, y, prob.cost_kind, prob.normalize_max)
            K = uot.kernel_from_cost(C, prob.eps, torch.float32)
            del C
            return uot.sinkhorn(a, b, K, m=prob.m, eps=prob.eps, tau=prob.tau, max_iter=T_)

        def timed(fn, T_):
            fn(3)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record()
            r = fn(T_)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1), r

        ms_on, r_on = timed(online, T)
        ms_on2, _ = timed(online, 2 * T)
        ms_st, r_st = timed(streamed, T)
        ms_st2, _ = timed(streamed, 2 * T)
        assert r_on.info()["flags"] == 0 and r_st.info()["flags"] == 0
        it_on = (ms_on2 - ms_on) / T * 1e3
        it_st = (ms_st2 - ms_st) / T * 1e3
        ent = prob.n * prob.m
        eps_ach = ent / (it_on * 1e-6)
        peak = LANE_SLOTS_PER_S / slots
        du = float(np.max(np.abs(r_on.u.cpu().numpy() / r_st.u.cpu().numpy() - 1.0)))
        out[key] = {
            "workload": f"{prob.n}x{prob.m} {d}-D points, eps={prob.eps}, tau={prob.tau}, {T} iterations",
            "solve_ms": round(ms_on, 3), "streamed_fp32_solve_ms": round(ms_st, 3),
            "iter_us": round(it_on, 2), "streamed_fp32_iter_us": round(it_st, 2),
            "speedup_solve_over_streamed": round(ms_st / ms_on, 3),
            "u_rel_diff_vs_streamed": float(f"{du:.3e}"),
            "roofline": {"bound": "alu", "achieved": round(eps_ach / 1e9, 1), "peak": round(peak / 1e9, 1),
                         "unit": "Gentries/s", "frac": round(eps_ach / peak, 4),
                         "slots_per_entry": slots, "traffic": None},
        }
    return out


def _events(torch, n=2):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def batched(uot, workloads, torch, dev, args):
    """Batching workload: 1024 problems, n, m ~ U[16, 2048], 300-D cosine,
    FP32 K (built before the timed region), 200 iterations, one persistent
    launch per solve (replayed from a HIP graph).  Compared with the plain
    FP32 form on the same GPU: the same problems solved one by one with the
    single-problem fused path (a sample, scaled by work)."""
    import numpy as np
    probs = workloads.batched()
    Ks, As, Bs = [], [], []
    for p in probs:
        C = uot.cost_from_points(torch.from_numpy(p.x).to(dev), torch.from_numpy(p.y).to(dev), p.cost_kind)
        Ks.append(uot.kernel_from_cost(C, p.eps, torch.float32))
        del C
        As.append(torch.from_numpy(p.a).to(dev))
        Bs.append(torch.from_numpy(p.b).to(dev))
    T = probs[0].max_iter
    solver = uot.BatchedSolver(Ks, As, Bs, eps=probs[0].eps, tau=probs[0].tau, max_iter=T, tune=1, trace=True)
    solver.run()
    torch.cuda.synchronize()
    tail = solver.tail_idle_fraction()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        solver.run()
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(g):
        solver.run()
    reps = max(min(args.steps, 5), 1)
    e0, e1 = _events(torch)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flags = [solver.result().info(i)["flags"] for i in (0, len(probs) - 1)]
    assert flags == [0, 0], flags
    elems = sum(p.n * p.m for p in probs)
    kbytes = elems * 4 * (T + 1)        # T iterations + the marginal sweep, K read once each
    # plain FP32 form: single-problem fused solves of a sample, scaled by work
    rng = np.random.default_rng(0)
    sample = rng.choice(len(probs), 32, replace=False)
    for i in sample[:2]:
        uot.sinkhorn(As[i], Bs[i], Ks[i], m=probs[i].m, eps=probs[i].eps, tau=probs[i].tau, max_iter=T)
    torch.cuda.synchronize()
    e0.record()
    for i in sample:
        uot.sinkhorn(As[i], Bs[i], Ks[i], m=probs[i].m, eps=probs[i].eps, tau=probs[i].tau, max_iter=T)
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1) * elems / sum(probs[i].n * probs[i].m for i in sample)
    return {"workload": f"batching: {len(probs)} problems, n,m ~ U[16,2048], 300-D cosine, FP32 K, eps=0.05, "
                        f"tau=1, {T} iterations, one persistent launch (HIP graph replay)",
            "ms_per_solve": round(ms, 3), "problem_iters_per_s": round(len(probs) * T / (ms * 1e-3), 1),
            "k_bytes_tb_s": round(kbytes / (ms * 1e-3) / 1e12, 3), "tail_idle_fraction": round(tail, 4),
            "split_problems": solver.nsplit, "queue_entries": solver.items,
            "plain_one_by_one_ms_est": round(single_ms, 1),
            "speedup_over_one_by_one": round(single_ms / ms, 2)}


def multi(uot, workloads, torch, dev, args):
    """Shared 8192^2 cosine kernel, 256 histogram pairs, 200 iterations on
    the matrix cores (BF16 K with hi/lo right-hand sides, and FP32 K).
    Algorithmic work 2 products x 2 n m R flops per iteration.  Compared
    with the plain FP32 form: single-pair fused solves on the same GPU."""
    base, A, B = workloads.multi_rhs()
    C = uot.cost_from_points(torch.from_numpy(base.x).to(dev), torch.from_numpy(base.y).to(dev), base.cost_kind)
    At = torch.from_numpy(A.T.copy()).to(dev)
    Bt = torch.from_numpy(B.T.copy()).to(dev)
    T = base.max_iter
    R = A.shape[1]
    flops = 2 * 2.0 * base.n * base.m * R
    out = {"workload": f"multi-RHS: shared {base.n}x{base.m} cosine kernel, R={R} pairs Dirichlet(0.5), "
                       f"eps=0.05, tau=1, {T} iterations", "flops_per_iter": flops}
    for name, dt in (("bf16", torch.bfloat16), ("f32", torch.float32)):
        K = uot.kernel_from_cost(C, base.eps, dt)
        variants = (("", 0), ("_lds128", 1), ("_direct", 2), ("_tiled128", 4)) if name == "bf16" else (("", 0),)
        for variant, tune in variants:
            uot.sinkhorn_multi(K, At, Bt, m=base.m, eps=base.eps, tau=base.tau, max_iter=2, tune=tune)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record()
            r = uot.sinkhorn_multi(K, At, Bt, m=base.m, eps=base.eps, tau=base.tau, max_iter=T, tune=tune)
            e1.record()
            torch.cuda.synchronize()
            assert r.info()["flags"] == 0
            ms = e0.elapsed_time(e1)
            out[name + variant] = {"ms_per_solve": round(ms, 3), "ms_per_iter": round(ms / T, 4),
                                   "tflop_s": round(flops * T / (ms * 1e-3) / 1e12, 2),
                                   "pair_iters_per_s": round(R * T / (ms * 1e-3), 1)}
        del K
    K = uot.kernel_from_cost(C, base.eps, torch.float32)
    a0, b0 = At[0].contiguous(), Bt[0].contiguous()
    uot.sinkhorn(a0, b0, K, m=base.m, eps=base.eps, tau=base.tau, max_iter=10)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for r in range(4):
        uot.sinkhorn(At[r].contiguous(), Bt[r].contiguous(), K, m=base.m, eps=base.eps, tau=base.tau, max_iter=T)
    e1.record()
    torch.cuda.synchronize()
    single = e0.elapsed_time(e1) / 4 * R
    out["plain_fp32_one_pair_at_a_time_ms_est"] = round(single, 1)
    out["speedup_bf16_over_plain"] = round(single / out["bf16"]["ms_per_solve"], 2)
    out["speedup_f32_over_plain"] = round(single / out["f32"]["ms_per_solve"], 2)
    return out


def precision(uot, workloads, torch, dev, args):
    """Precision workload at full size (65536 x 8192, eps 1e-3, absorption
    above 30 checked every 10 iterations, 2000 iterations) with the kernel
    stored in FP32, BF16 and FP8; iterations/s and K stream rate of each."""
    prob = workloads.precision()
    C = uot.cost_from_points(torch.from_numpy(prob.x).to(dev), torch.from_numpy(prob.y).to(dev),
                             prob.cost_kind, prob.normalize_max)
    a = torch.from_numpy(prob.a).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    out = {"workload": f"precision: {prob.n}x{prob.m}, 16-D normal points, eps={prob.eps}, tau={prob.tau}, "
                       f"{prob.max_iter} iterations, absorption at |log| > 30 checked every 10 iterations "
                       "(FP8: every 2)"}
    ref = _load_precision_ref(prob)
    for name, dt, eb in (("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2), ("fp8", torch.float8_e4m3fn, 1)):
        e0, e1 = _events(torch)
        e0.record()
        r = uot.sinkhorn(a, b, None, C=C, k_dtype=dt, eps=prob.eps, tau=prob.tau, max_iter=prob.max_iter,
                         absorb_log_threshold=30.0, check_every=2 if name == "fp8" else 10, profile=True)
        e1.record()
        torch.cuda.synchronize()
        info = r.info()
        ms = e0.elapsed_time(e1)
        p = r.profile
        pass_us = p["fused_ms"] * 1e3 / max(p["fused_launches"], 1)
        out[name] = {"ms_per_solve": round(ms, 2), "iters_per_s": round(prob.max_iter / (ms * 1e-3), 1),
                     "pass_us": round(pass_us, 2), "pass_tb_s": round(prob.n * prob.m * eb / (pass_us * 1e-6) / 1e12, 3),
                     "absorptions": info["absorptions"], "flags": info["flags"]}
        if ref is not None:
            out[name]["err_vs_oracle"] = _precision_errors(r.f.cpu().numpy(), r.g.cpu().numpy(),
                                                           float(r.loss.cpu()), ref, prob.eps)
    if ref is None:
        out["err_vs_oracle"] = f"missing {PRECISION_REF}"
    return out


def log_domain(uot, workloads, torch, dev, args):
    """Log-domain solve on the precision workload (65536 x 8192, eps 1e-3,
    tau 0.1, 2000 iterations): the cost read as FP64 (8 bytes per entry and
    iteration) and as FP32 (4), no absorption; iterations/s, the pass's cost
    stream rate (per-iteration time from two solves of T and 2T iterations,
    pass plus column finalize) and the errors against the FP64 oracle.  Then
    eps-scaling: the same problem to tol 1e-5 directly and from eps0 = 0.064
    (halving, 20 iterations per stage), iterations and time of each."""
    prob = workloads.precision()
    C = uot.cost_from_points(torch.from_numpy(prob.x).to(dev), torch.from_numpy(prob.y).to(dev),
                             prob.cost_kind, prob.normalize_max)
    a = torch.from_numpy(prob.a).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    ref = _load_precision_ref(prob)
    out = {"workload": f"precision: {prob.n}x{prob.m}, 16-D normal points, eps={prob.eps}, tau={prob.tau}, "
                       f"{prob.max_iter} iterations, log-domain passes over the stored cost"}

    def timed(T, **kw):
        e0, e1 = _events(torch)
        e0.record()
        r = uot.sinkhorn_lse(C, a, b, eps=prob.eps, tau=prob.tau, max_iter=T, **kw)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), r

    for name, dt, eb in (("f64_cost", torch.float64, 8), ("f32_cost", torch.float32, 4)):
        timed(3, cost_dtype=dt)
        ms1, _ = timed(100, cost_dtype=dt)
        ms2, _ = timed(200, cost_dtype=dt)
        it_us = (ms2 - ms1) / 100 * 1e3
        ms, r = timed(prob.max_iter, cost_dtype=dt)
        info = r.info()
        out[name] = {"ms_per_solve": round(ms, 2), "iters_per_s": round(prob.max_iter / (ms * 1e-3), 1),
                     "iter_us": round(it_us, 2), "cost_tb_s": round(prob.n * prob.m * eb / (it_us * 1e-6) / 1e12, 3),
                     "hbm_frac": round(prob.n * prob.m * eb / (it_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "flags": info["flags"]}
        if ref is not None:
            out[name]["err_vs_oracle"] = _precision_errors(r.f.cpu().numpy(), r.g.cpu().numpy(), float(r.loss.cpu()),
                                                           ref, prob.eps)
    sched = {"direct": {}, "eps_scaled": {"eps0": 0.064, "factor": 0.5, "stage_iters": 20}}
    out["to_tol_1e-5"] = {}
    for name, kw in sched.items():
        ms, r = timed(20000, tol=1e-5, check_every=10, **kw)
        info = r.info()
        out["to_tol_1e-5"][name] = {"iters": info["iters"], "ms": round(ms, 2), "err": float(f"{info['err']:.3e}"),
                                    "flags": info["flags"]}
    return out


PRECISION_REF = os.path.join(ROOT, "tests", "golden", "precision_65536x8192_fp64.npz")


def _load_precision_ref(prob):
    """The FP64 oracle's result at the precision workload's full size, stored
    by tests/golden/make_precision_reference.py."""
    import numpy as np
    if not os.path.exists(PRECISION_REF):
        return None
    z = np.load(PRECISION_REF)
    if int(z["n"]) != prob.n or int(z["m"]) != prob.m or int(z["iters"]) != prob.max_iter:
        return None
    return {k: z[k] for k in z.files}


def _precision_errors(f, g, loss, ref, eps):
    """u, v errors from the potentials (entrywise max |u/u_ref - 1|, and
    normwise ||U - U_ref|| / ||U_ref|| with U scaled by its largest entry)
    and the relative loss error."""
    import numpy as np
    out = {}
    for name, x, x0 in (("u", f, ref["f"]), ("v", g, ref["g"])):
        d = np.expm1((x - x0) / eps)
        w = np.exp((x0 - x0.max()) / eps)
        out[name + "_entrywise"] = float(f"{np.max(np.abs(d)):.3e}")
        out[name + "_normwise"] = float(f"{np.linalg.norm(d * w) / np.linalg.norm(w):.3e}")
    L0 = float(ref["loss"])
    out["loss"] = float(f"{abs(loss - L0) / abs(L0):.3e}")
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(threads: int, rows: int, reps: int) -> None:
    """Child process of cpu_baseline: the FP64 oracle on the headline recipe
    with ``rows`` source points and ``threads`` OpenMP threads bound to
    cores; prints the per-run rates (iterations/s of that sample) as JSON."""
    import oracle
    import workloads
    prob = workloads.headline(n=rows)
    C = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    K = oracle.kernel(C, prob.eps)
    del C
    T1 = 2
    rates = []
    for _ in range(reps):
        a0 = time.perf_counter()
        oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T1)
        d1 = time.perf_counter() - a0
        T2 = T1 + max(5, int(3.0 / max(d1 / T1, 1e-3)))
        b0 = time.perf_counter()
        oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T2)
        d2 = time.perf_counter() - b0
        rates.append((T2 - T1) / (d2 - d1))
    print(json.dumps({"rates": rates, "T2": T2}), flush=True)


def cpu_baseline(prob):
    """FP64 oracle on the host cores, in child processes (OpenMP threads
    bound one per core, OMP_PROC_BIND=close, OMP_PLACES=cores): the headline
    workload at full size on every core this process may run on (median of
    3 runs), and on one core at 2048 x 16384 (the same recipe with 1/8 of
    the rows; the rate is scaled to the full size).  Each run times T1 and T2
    iterations of the plain loop, kernel built beforehand, and takes
    (T2 - T1) / (time2 - time1), which cancels per-call setup."""
    import statistics
    import subprocess
    avail = len(os.sched_getaffinity(0))
    cores = min(avail, int(os.environ.get("OMP_NUM_THREADS", avail)))

    def leg(threads, rows, reps):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PROC_BIND="close", OMP_PLACES="cores")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", str(threads), "--cpu-rows",
                            str(rows), "--cpu-reps", str(reps)], env=env, capture_output=True, text=True,
                           timeout=600)
        if r.returncode != 0:
            raise RuntimeError(f"cpu leg failed: {r.stderr[-2000:]}")
        return json.loads(r.stdout.strip().splitlines()[-1])

    t0 = time.perf_counter()
    multi = leg(cores, prob.n, 3)
    one = leg(1, 2048, 1)
    wall = time.perf_counter() - t0
    rate = statistics.median(multi["rates"])
    rate1 = one["rates"][0] * 2048 / prob.n
    return {"value": round(rate, 3), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "runs": [round(x, 3) for x in multi["rates"]], "one_core_value": round(rate1, 4),
            "cpu_model": _cpu_model(), "omp": "OMP_PROC_BIND=close OMP_PLACES=cores",
            "sample": f"headline workload at full size ({prob.n}x{prob.m}, FP64 K): median of 3 runs, each a "
                      f"{multi['T2']}-iteration run minus a 2-iteration run (kernel build excluded); one core: "
                      f"2048 x {prob.m}, {one['T2']} minus 2 iterations, scaled by 2048/{prob.n}; wall {wall:.1f} s"}


if __name__ == "__main__":
    main()
