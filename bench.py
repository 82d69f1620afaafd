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
  plain         the plain two-pass form on the same GPU (same steps).
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
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU: every box here has a single MI355X "
                 "(--gpus must be 1; the multi-GPU sharding is described in DESIGN.md)")
    import numpy as np
    import torch

    import paper_2412_11079_amd as uot
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)

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
    if not args.no_grad:
        out["fwd_bwd"] = fwd_bwd(uot, workloads, torch, dev, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


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
        ga, gb, gx = uot.sinkhorn_backward(r, g, x=x, y=y)
        e2.record()
        torch.cuda.synchronize()
        f_ms += e0.elapsed_time(e1)
        b_ms += e1.elapsed_time(e2)
    f_ms /= reps
    b_ms /= reps
    kb = prob.n * prob.m * 4
    # forward: T passes; reverse: T recompute + T adjoint passes + 1 column + 1 seed pass
    passes = prob.max_iter * 3 + 3
    return {"workload": f"grad: N=M={prob.n} FP32 K, {prob.max_iter} iterations, checkpoints every "
                        f"{prob.checkpoint_every}, gradients for x, a, b",
            "fwd_ms": round(f_ms, 3), "bwd_ms": round(b_ms, 3), "fwd_bwd_ms": round(f_ms + b_ms, 3),
            "k_passes": passes, "k_bytes_tb_s": round(passes * kb / ((f_ms + b_ms) * 1e-3) / 1e12, 3)}


def cpu_baseline(prob):
    """FP64 oracle on the host cores: kernel built once (untimed), then two
    runs of T1 and T2 iterations; the rate is (T2 - T1) / (t2 - t1)."""
    import numpy as np

    import oracle
    C = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    K = oracle.kernel(C, prob.eps)
    del C
    T1, T2 = 2, 12
    t0 = time.perf_counter()
    oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T1)
    t1 = time.perf_counter()
    oracle.sinkhorn(K, prob.a, prob.b, prob.eps, prob.tau, T2)
    t2 = time.perf_counter()
    rate = (T2 - T1) / ((t2 - t1) - (t1 - t0))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(rate, 3), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"headline workload at full size ({prob.n}x{prob.m}, FP64 K), {T2}-iteration run minus "
                      f"{T1}-iteration run (kernel build excluded); wall {t2 - t0:.1f} s"}


if __name__ == "__main__":
    main()
