"""Write the oracle's results on a full-size workload to <workload>_oracle.json.

Calls only oracle/ and workloads.py.  Stored: the rank profiles of both
phases, and the products G x, Z x and X (Y x) for two seeded Gaussian probe
vectors sampled at 512 seeded positions (cluster order), plus their full
norms.  Run: python tests/golden/make_golden.py c2   (or c3)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

NAMES = {"c2": W.C2, "c3": W.C3}


def main(key: str):
    w = NAMES[key]
    pts = w.points()
    t0 = time.time()
    tree, bt, X, Y = O.build_problem(pts, w.leaf_size, w.eta, w.order, w.kernel_x, w.kernel_y)
    print(f"[{key}] problem built ({time.time() - t0:.1f}s)", flush=True)
    p1, p2 = O.multiply(X, Y, bt, w.eps)
    elapsed = time.time() - t0
    print(f"[{key}] oracle done ({elapsed:.1f}s)", flush=True)
    x = W.probe_vectors(101, w.n, 2)
    idx = np.sort(np.random.default_rng(102).choice(w.n, 512, replace=False))
    gx, zx, xyx = p1.G.matvec(x), p2.Z.matvec(x), X.matvec(Y.matvec(x))
    nc = tree.nclusters
    out = {
        "workload": w.name, "eps": w.eps, "oracle_seconds": elapsed,
        "probe_seed": 101, "index_seed": 102, "index": idx.tolist(),
        "ranks_p1_row": [int(p1.row.Q.rank[c]) for c in range(nc)],
        "ranks_p1_col": [int(p1.col.Q.rank[c]) for c in range(nc)],
        "ranks_p2_row": [int(p2.row.Q.rank[c]) for c in range(nc)],
        "ranks_p2_col": [int(p2.col.Q.rank[c]) for c in range(nc)],
        "Gx": gx[idx].tolist(), "Zx": zx[idx].tolist(), "XYx": xyx[idx].tolist(),
        "Gx_norm": np.linalg.norm(gx, axis=0).tolist(), "Zx_norm": np.linalg.norm(zx, axis=0).tolist(),
        "XYx_norm": np.linalg.norm(xyx, axis=0).tolist(),
        "txy_adm": len(p1.G.S), "txy_inadm": len(p1.G.N),
    }
    with open(os.path.join(HERE, f"{key}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote {key}_oracle.json (oracle {elapsed:.1f}s)")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
