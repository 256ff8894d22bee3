"""Write the oracle's results on a full-size workload to <workload>_oracle.json.

Calls only oracle/ and workloads.py.  Run:
    python tests/golden/make_golden.py c2      (or c3, dlp, c5s, or c4)

dlp is the double-layer recipe at n = 49152 (the oracle's memory at
n = 110592 exceeds what the generating host holds); c5s is the recipe of
the cube workload (1/r, k = 64) at n = 16384.

For the single-product workloads (c2, c3, dlp) the file holds
  - the rank profiles of both phases (row and column bases);
  - a two-sided randomized sketch of G, Z and X Y:  Psi^T M Omega with
    Omega = probe_vectors(101, n, 32) and Psi = probe_vectors(103, n, 32)
    (independent Gaussian matrices); ||Psi^T (A - B) Omega||_F estimates
    sqrt(32 * 32) ||A - B||_F, so ratios of sketch norms estimate relative
    Frobenius distances over all n^2 entries, and column j of the sketch
    estimates the relative distance of the products with probe j;
  - the norms ||M omega_j|| of those products (all n entries);
  - the products with the first two probes at 512 seeded positions;
  - the relative spectral error ||Z - X Y||_2 / ||X Y||_2 of the oracle's Z
    by 20 steps of power iteration from probe_vectors(104, n, 1);
  - the oracle's algorithmic work per step and kind (the ledger of
    oracle.counting()) and its wall time on the generating host.

For the batched workload (c4: 64 independent products) the file holds per
instance the per-level sums of the four rank profiles, a SHA-256 digest of
the profiles, Z x at 32 seeded positions with its norms, and 8 x 8 sketches
of G and Z (8 probes, 8 sketch rows: seeds 700 + i and 800 + i).
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

NAMES = {"c2": W.C2, "c3": W.C3, "dlp": W.C6S, "c5s": W.C5S}
PROBE_SEED, SKETCH_SEED, INDEX_SEED, POWER_SEED = 101, 103, 102, 104
NPROBE = 32
POWER_STEPS = 20


def power_error(Z, X, Y, n, seed, steps):
    """||Z - X Y||_2 / ||X Y||_2, each norm by `steps` power iterations on
    A^T A from the same seeded start vector (Section 7 reports this error)."""
    def norm2(apply, applyT):
        v = W.probe_vectors(seed, n, 1)
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(steps):
            w = applyT(apply(v))
            lam = float(np.linalg.norm(w))
            if lam == 0.0:
                return 0.0
            v = w / lam
        return np.sqrt(lam)
    Zt, Xt, Yt = Z.transposed(), X.transposed(), Y.transposed()
    e = norm2(lambda v: Z.matvec(v) - X.matvec(Y.matvec(v)), lambda v: Zt.matvec(v) - Yt.matvec(Xt.matvec(v)))
    r = norm2(lambda v: X.matvec(Y.matvec(v)), lambda v: Yt.matvec(Xt.matvec(v)))
    return e / r


def ledger_table(led):
    out = {}
    for (step, kind), v in led.items():
        out.setdefault(step, {})[kind] = v
    return out


def main(key: str):
    w = NAMES[key]
    pts = w.points()
    t0 = time.time()
    tree, bt, X, Y = O.build_problem(pts, w.leaf_size, w.eta, w.order, w.kernel_x, w.kernel_y,
                                     normals=w.normals())
    t1 = time.time()
    print(f"[{key}] problem built ({t1 - t0:.1f}s)", flush=True)
    with O.counting() as led:
        p1, p2 = O.multiply(X, Y, bt, w.eps)
    elapsed = time.time() - t1
    print(f"[{key}] oracle done ({elapsed:.1f}s)", flush=True)
    om = W.probe_vectors(PROBE_SEED, w.n, NPROBE)
    psi = W.probe_vectors(SKETCH_SEED, w.n, NPROBE)
    idx = np.sort(np.random.default_rng(INDEX_SEED).choice(w.n, 512, replace=False))
    gx, zx, xyx = p1.G.matvec(om), p2.Z.matvec(om), X.matvec(Y.matvec(om))
    print(f"[{key}] probes done", flush=True)
    eps2 = power_error(p2.Z, X, Y, w.n, POWER_SEED, POWER_STEPS)
    print(f"[{key}] power iteration done: eps2 = {eps2:.3e}", flush=True)
    nc = tree.nclusters
    out = {
        "workload": w.name, "eps": w.eps, "oracle_seconds": elapsed,
        "oracle_threads": _threads(),
        "probe_seed": PROBE_SEED, "sketch_seed": SKETCH_SEED, "nprobe": NPROBE,
        "index_seed": INDEX_SEED, "index": idx.tolist(),
        "ranks_p1_row": [int(p1.row.Q.rank[c]) for c in range(nc)],
        "ranks_p1_col": [int(p1.col.Q.rank[c]) for c in range(nc)],
        "ranks_p2_row": [int(p2.row.Q.rank[c]) for c in range(nc)],
        "ranks_p2_col": [int(p2.col.Q.rank[c]) for c in range(nc)],
        "sketch_G": (psi.T @ gx).tolist(), "sketch_Z": (psi.T @ zx).tolist(),
        "sketch_XY": (psi.T @ xyx).tolist(),
        "Gx_norm": np.linalg.norm(gx, axis=0).tolist(), "Zx_norm": np.linalg.norm(zx, axis=0).tolist(),
        "XYx_norm": np.linalg.norm(xyx, axis=0).tolist(),
        "Gx": gx[idx, :2].tolist(), "Zx": zx[idx, :2].tolist(), "XYx": xyx[idx, :2].tolist(),
        "power_seed": POWER_SEED, "power_steps": POWER_STEPS, "eps2_Z": eps2,
        "txy_adm": len(p1.G.S), "txy_inadm": len(p1.G.N),
        "ledger": ledger_table(led),
    }
    with open(os.path.join(HERE, f"{key}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote {key}_oracle.json (oracle {elapsed:.1f}s)")


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return None


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
    for i, (w, pts) in enumerate(W.batched_instances()):
        t0 = time.time()
        tree, bt, X, Y = O.build_problem(pts, w.leaf_size, w.eta, w.order, w.kernel_x, w.kernel_y)
        p1, p2 = O.multiply(X, Y, bt, w.eps)
        nc = tree.nclusters
        prof = [[int(p.Q.rank[c]) for c in range(nc)] for p in (p1.row, p1.col, p2.row, p2.col)]
        x = W.probe_vectors(w.seed + 500, w.n, 2)
        idx = np.sort(np.random.default_rng(w.seed + 600).choice(w.n, 32, replace=False))
        zx = p2.Z.matvec(x)
        om = W.probe_vectors(700 + i, w.n, 8)
        psi = W.probe_vectors(800 + i, w.n, 8)
        out["instances"].append({
            "name": w.name, "n": w.n, "order": w.order, "eps": w.eps,
            "probe_seed": w.seed + 500, "index": idx.tolist(),
            "rank_digest": rank_digest(prof), "level_sums": [level_sums(tree, p) for p in prof],
            "Zx": zx[idx].tolist(), "Zx_norm": np.linalg.norm(zx, axis=0).tolist(),
            "sketch_probe_seed": 700 + i, "sketch_seed": 800 + i,
            "sketch_G": (psi.T @ p1.G.matvec(om)).tolist(), "sketch_Z": (psi.T @ p2.Z.matvec(om)).tolist(),
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
