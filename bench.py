"""Benchmark of the adaptive H^2 product Z = X Y on one MI355X.

One step is the whole hot path on the 2-D workload (n = 16384 points in the
unit square, X = log|x-y|, Y = exp(-|x-y|), leaf 64, eta 1, Chebyshev order
4 -> k = 16, eps = 1e-6): phase 1 (h2_mul_intermediate: induced bases and G
on T^XY) and phase 2 (h2_recompress into Z's block tree).  Inputs (tree,
X, Y) are resident on the GPU before timing.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision both|fp64|fp32]
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


FAMILY_KERNELS = {"gemm_sum": ("gemm_sum_kernel", "gemm_tri_kernel", "gemm_tri_block_kernel", "chain3_kernel"),
                  "tsqr": ("tsqr_rb_kernel", "tsqr_kernel"),
                  "jacobi": ("jacobi_kernel", "jacobi_small_kernel")}


def measured_traffic(family: str, precision: str):
    """HBM bytes per launch of a kernel family from the committed counter
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when the summary is
    missing or the kernels changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_2d_n16384_{precision}.md")
    src = os.path.join(ROOT, "paper_2309_09061_amd", "csrc", "kernels_la.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernels source sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    launches = total = 0.0
    for row in re.finditer(r"^\| ([^|]+) \| (\d+) \| ([0-9.]+) \| ([0-9.]+) \|$", text, re.M):
        name = row.group(1).split("<")[0].strip()
        if name in FAMILY_KERNELS.get(family, ()):
            n = float(row.group(2))
            launches += n
            total += n * (float(row.group(3)) + float(row.group(4))) * 2**20
    return total / launches if launches else None


def copy_calibration():
    """A plain device copy of 2^25 float64 (256 MiB read, 256 MiB written):
    the counters FETCH_SIZE / WRITE_SIZE of this copy against its known bytes
    give the scale applied to the counters of the library kernels."""
    import torch
    a = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {a.numel() * 8} bytes", flush=True)


def run_form(ctx, T, X, Y, w, precision, steps, warmup, families=None):
    """Warm-up, then `steps` timed steps of the hot path in one precision;
    launches of the kernel families named in `families` (all when None) are
    timed with HIP events inside the timed region."""
    import torch

    from paper_2309_09061_amd import h2

    def step():
        G = h2.h2_mul_intermediate(ctx, X, Y, w.eps, precision)
        Z = h2.h2_recompress(ctx, G, h2.Matrix.zero(ctx, T), w.eps, precision)
        return G, Z

    for i in range(warmup):
        G, Z = step()
        torch.cuda.synchronize()
        print(f"[{precision}] warmup step {i + 1}/{warmup} done", file=sys.stderr, flush=True)
        del G, Z
    ctx.profile(True, families)
    ctx.kernel_stats(reset=True)
    ctx.step_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        G, Z = step()
        if i < steps - 1:
            del G, Z
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dev = ctx.step_times()
    host = ctx.step_times(host=True, reset=True)
    ks = ctx.kernel_stats()
    ctx.profile(False)
    print(f"[{precision}] {steps} timed steps done ({'all' if families is None else ','.join(families)} "
          f"kernel families timed)", file=sys.stderr, flush=True)
    return {"ms": (t1 - t0) / steps * 1e3, "dev": {k: v / steps for k, v in dev.items()},
            "host": {k: v / steps for k, v in host.items()}, "ks": ks, "G": G, "Z": Z, "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32"],
                    help="fp64: the float64 form; fp32: bulk products in float32; both: "
                         "the float64 form as the headline value, the mixed form beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB on the GPU (the reference for the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design note, not a run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2309_09061_amd import h2

    w = W.C2
    ctx = h2.Context(0)
    T = h2.Tree(ctx, w.points(), w.leaf_size, w.eta)
    X = h2.Matrix.kernel(ctx, T, w.kernel_x, w.order)
    Y = h2.Matrix.kernel(ctx, T, w.kernel_y, w.order)
    torch.cuda.synchronize()

    main_prec = "fp32" if args.precision == "fp32" else "fp64"
    # breakdown run: every launch timed (the events add host time per launch),
    # giving the per-family kernel time and the dominant family
    nb = max(2, min(args.steps, 3))
    br = run_form(ctx, T, X, Y, w, main_prec, nb, args.warmup)
    bks = br["ks"]
    dom = max(bks, key=lambda k: bks[k]["ms"])
    del br
    # headline run: only the dominant family's launches carry events
    r = run_form(ctx, T, X, Y, w, main_prec, args.steps, 1, families=[dom])
    G, Z, ks, ms = r["G"], r["Z"], r["ks"], r["ms"]
    ranks = {"p1_row_max": int(G.ranks(0).max()), "p2_row_max": int(Z.ranks(0).max()),
             "p2_row_mean": float(Z.ranks(0).mean())}
    sizes = G.sizes()

    d = ks[dom]
    mfma_peak = PEAK["fp64_mfma" if main_prec == "fp64" else "fp32_mfma"]
    if dom == "gemm_sum":
        bound, peak = "mfma", mfma_peak
    else:
        bound, peak = "alu", PEAK["fp64_vector"]
    achieved = d["flops"] / (d["ms"] * 1e-3) if d["ms"] > 0 else 0.0
    gemm = bks["gemm_sum"]
    mfma_util = gemm["flops"] / nb / (ms * 1e-3) / mfma_peak

    out = {
        "metric": "H^2 product time (s) and MFMA util at eps; mixed vs FP64 on one MI355X",
        "value": ms * 1e-3, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32-bulk/f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "leaf": w.leaf_size, "eta": w.eta,
                   "order": w.order, "rank": w.rank, "kernel_x": w.kernel_x, "kernel_y": w.kernel_y,
                   "eps": w.eps, "precision": main_prec},
        "roofline": {"kernel": dom, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(dom, main_prec),
                     "avg_launch_ms": d["ms"] / max(d["launches"], 1),
                     "flops_per_launch": d["flops"] / max(d["launches"], 1)},
        "mfma_util_step": mfma_util,
        "kernel_ms_per_step": {k: v["ms"] / nb for k, v in bks.items()},
        "kernel_ms_per_step_note": f"from {nb} further steps with every launch timed",
        "step_ms": r["dev"],
        "host_step_ms": r["host"],
        "ranks": ranks, "product_tree": sizes,
    }
    if args.precision == "both":
        m = run_form(ctx, T, X, Y, w, "fp32", args.steps, args.warmup, families=["gemm_sum"])
        # distance of the mixed Z to the float64 Z on seeded probe vectors
        x = torch.from_numpy(np.ascontiguousarray(W.probe_vectors(7, w.n, 2).T)).cuda().t()
        z64 = torch.zeros((2, w.n), dtype=torch.float64, device="cuda").t()
        z32 = torch.zeros((2, w.n), dtype=torch.float64, device="cuda").t()
        Z.matvec(x, z64)
        m["Z"].matvec(x, z32)
        torch.cuda.synchronize()
        diff = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
        mg = m["ks"]["gemm_sum"]
        out["mixed"] = {"precision": "fp32 bulk products, fp64 factorizations", "ms_per_step": m["ms"],
                        "speedup_vs_fp64": ms / m["ms"], "rel_diff_Zx_vs_fp64": diff,
                        "gemm_ms_per_step": mg["ms"] / m["steps"],
                        "mfma_util_step": mg["flops"] / m["steps"] / (m["ms"] * 1e-3) / PEAK["fp32_mfma"],
                        "step_ms": m["dev"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
