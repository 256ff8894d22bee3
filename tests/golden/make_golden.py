"""Write the oracle's results on a full-size workload to <workload>_oracle.json.

Calls only oracle/ and workloads.py.  Stored: the rank profiles of both
phases, and the products G x, Z x and X (Y x) for two seeded Gaussian probe
vectors sampled at 512 seeded positions (cluster order), plus their full
norms.  Run: python tests/golden/make_golden.py c2   (or c3)

For the batched workload (c4: 64 independent products) the file holds, per
instance, the per-level sums of the four rank profiles, a SHA-256 digest of
the profiles themselves, and Z x sampled at 32 seeded positions with its
norms.  Run: python tests/golden/make_golden.py c4
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


def rank_digest(profiles) -> str:
    """SHA-256 of the four rank profiles (int32, row p1, col p1, row p2, col p2)."""
    import hashlib
    h = hashlib.sha256()
    for p in profiles:
        h.update(np.asarray(p, dtype=np.int32).tobytes())
    return h.hexdigest()


def level_sums(tree, ranks):
    return [int(sum(ranks[c] for c in tree.clusters_at(lev))) for lev in range(tree.depth + 1)]


def main_batched():
    out = {"workload": "c4_batched_64", "instances": []}
    t00 = time.time()
    for w, pts in W.batched_instances():
        t0 = time.time()
        tree, bt, X, Y = O.build_problem(pts, w.leaf_size, w.eta, w.order, w.kernel_x, w.kernel_y)
        p1, p2 = O.multiply(X, Y, bt, w.eps)
        nc = tree.nclusters
        prof = [[int(p.Q.rank[c]) for c in range(nc)] for p in (p1.row, p1.col, p2.row, p2.col)]
        x = W.probe_vectors(w.seed + 500, w.n, 2)
        idx = np.sort(np.random.default_rng(w.seed + 600).choice(w.n, 32, replace=False))
        zx = p2.Z.matvec(x)
        out["instances"].append({
            "name": w.name, "n": w.n, "order": w.order, "eps": w.eps,
            "probe_seed": w.seed + 500, "index": idx.tolist(),
            "rank_digest": rank_digest(prof), "level_sums": [level_sums(tree, p) for p in prof],
            "Zx": zx[idx].tolist(), "Zx_norm": np.linalg.norm(zx, axis=0).tolist(),
        })
        print(f"[c4] {w.name} n={w.n} order={w.order} ({time.time() - t0:.1f}s)", flush=True)
    out["oracle_seconds"] = time.time() - t00
    with open(os.path.join(HERE, "c4_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote c4_oracle.json (oracle {out['oracle_seconds']:.1f}s)")


if __name__ == "__main__":
    key = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if key == "c4":
        main_batched()
    else:
        main(key)
