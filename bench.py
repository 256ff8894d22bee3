"""Benchmark of the adaptive H^2 product Z = X Y on one MI355X.

One step is the whole hot path on the 2-D workload (n = 16384 points in the
unit square, X = log|x-y|, Y = exp(-|x-y|), leaf 64, eta 1, Chebyshev order
4 -> k = 16, eps = 1e-6): phase 1 (h2_mul_intermediate: induced bases and G
on T^XY) and phase 2 (h2_recompress into Z's block tree).  Inputs (tree,
X, Y) are resident on the GPU before timing.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK = {"fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "fp64_vector": 78.6e12, "hbm": 8.0e12}


def cpu_baseline(seconds_budget: float = 30.0):
    """The FP64 oracle on a bounded sample of the same workload: the same recipe
    (seeded points, kernels, leaf size, order, eps) at n = 4096, extrapolated
    linearly to n = 16384 (the method's cost is O(n))."""
    import numpy as np

    import oracle as O
    import workloads as W
    w = W.C2
    n_s = 4096
    pts = W.make_points(w.seed, n_s, w.dim, w.distribution)
    tree, bt, X, Y = O.build_problem(pts, w.leaf_size, w.eta, w.order, w.kernel_x, w.kernel_y)
    t0 = time.perf_counter()
    O.multiply(X, Y, bt, w.eps)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = 1
    return {"value": dt * w.n / n_s, "unit": "s", "cores": int(cores), "kind": "oracle",
            "sample": f"oracle phase 1 + phase 2 on the same recipe at n={n_s} ({dt:.2f} s), "
                      f"scaled by n={w.n}/{n_s} (linear complexity)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design note, not a run)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2309_09061_amd import h2

    w = W.C2
    ctx = h2.Context(0)
    T = h2.Tree(ctx, w.points(), w.leaf_size, w.eta)
    X = h2.Matrix.kernel(ctx, T, w.kernel_x, w.order)
    Y = h2.Matrix.kernel(ctx, T, w.kernel_y, w.order)
    torch.cuda.synchronize()

    def step():
        G = h2.h2_mul_intermediate(ctx, X, Y, w.eps, args.precision)
        Z = h2.h2_recompress(ctx, G, h2.Matrix.zero(ctx, T), w.eps, args.precision)
        return G, Z

    for i in range(args.warmup):
        G, Z = step()
        torch.cuda.synchronize()
        print(f"warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
        del G, Z
    ctx.profile(True)
    ctx.kernel_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, hsteps = {}, {}
    for i in range(args.steps):
        G, Z = step()
        for k, v in ctx.step_times().items():
            steps[k] = steps.get(k, 0.0) + v
        for k, v in ctx.step_times(host=True).items():
            hsteps[k] = hsteps.get(k, 0.0) + v
        if i < args.steps - 1:
            del G, Z
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ks = ctx.kernel_stats()
    ctx.profile(False)
    ms = (t1 - t0) / args.steps * 1e3
    ranks = {"p1_row_max": int(G.ranks(0).max()), "p2_row_max": int(Z.ranks(0).max()),
             "p2_row_mean": float(Z.ranks(0).mean())}
    sizes = G.sizes()

    dom = max(ks, key=lambda k: ks[k]["ms"])
    d = ks[dom]
    if dom == "gemm_sum":
        bound, peak = "mfma", PEAK["fp64_mfma" if args.precision == "fp64" else "fp32_mfma"]
    else:
        bound, peak = "alu", PEAK["fp64_vector"]
    achieved = d["flops"] / (d["ms"] * 1e-3) if d["ms"] > 0 else 0.0
    gemm = ks["gemm_sum"]
    mfma_util = gemm["flops"] / (args.steps * ms * 1e-3) / PEAK["fp64_mfma"]

    out = {
        "metric": "H^2 product time (s) and MFMA util at eps; mixed vs FP64 on one MI355X",
        "value": ms * 1e-3, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-bulk/f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "leaf": w.leaf_size, "eta": w.eta,
                   "order": w.order, "rank": w.rank, "kernel_x": w.kernel_x, "kernel_y": w.kernel_y,
                   "eps": w.eps, "precision": args.precision},
        "roofline": {"kernel": dom, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_ms": d["ms"] / max(d["launches"], 1),
                     "flops_per_launch": d["flops"] / max(d["launches"], 1)},
        "mfma_util_step": mfma_util,
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in ks.items()},
        "step_ms": {k: v / args.steps for k, v in steps.items()},
        "host_step_ms": {k: v / args.steps for k, v in hsteps.items()},
        "ranks": ranks, "product_tree": sizes,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
