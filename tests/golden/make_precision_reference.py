"""Writes the FP64 reference of the precision workload at its full size
(65536 x 8192, 16-D standard-normal points, squared-Euclidean cost divided
by its maximum, Dirichlet(1) histograms, eps 1e-3, tau 0.1, 2000
iterations) to precision_65536x8192_fp64.npz beside this file.

Only the oracle computes it: the textbook stabilised iteration in FP64
(potentials absorbed whenever a scaling's log leaves [-30, 30]; in FP64
this is a reparameterisation of the plain iteration, which would leave the
FP64 range here since C/eps reaches 1000), then the plan's marginals and the
objective from the final potentials.  Stored: the potentials f = eps log u,
g = eps log v of the total scalings, the objective, and the iteration count.

Run: python tests/golden/make_precision_reference.py   (about 15 minutes on
8 cores, 9 GB of memory)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "precision_65536x8192_fp64.npz")


def main():
    prob = workloads.precision()
    t0 = time.time()
    C = oracle.cost_points(prob.x, prob.y, prob.cost_kind, prob.normalize_max)
    print(f"cost {C.shape} in {time.time() - t0:.1f} s", flush=True)
    f, g, nabs = oracle.sinkhorn_stabilized(C, prob.a, prob.b, prob.eps, prob.tau, prob.max_iter, 30.0)
    print(f"stabilised iteration ({nabs} absorptions) in {time.time() - t0:.1f} s", flush=True)
    r, c = oracle.potential_marginals(C, f, g, prob.eps)
    loss = oracle.loss_potentials(f, g, r, c, prob.a, prob.b, prob.eps, prob.tau)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g)) and np.isfinite(loss)
    np.savez(OUT, f=f, g=g, loss=np.float64(loss), iters=np.int64(prob.max_iter), n=np.int64(prob.n),
             m=np.int64(prob.m))
    print(f"loss {loss:.15e}; wrote {OUT} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
