"""Sanitizer builds of the host symbolic layer (no GPU).

tree.cpp (cluster tree, block tree and the product tree T^XY of Section 6,
whose wide levels are built on two host threads) is compiled with g++ twice
into a small driver: once with AddressSanitizer and UndefinedBehaviorSanitizer,
once with ThreadSanitizer.  Each build runs on seeded inputs and must finish
without a report, and its trees must equal the oracle's (cluster permutation
and offsets, block types, and the product tree's blocks with their triples).
The threaded sweep starts once a level holds 65536 middle triples; the 2-D
case at n = 16384 with leaf size 16 reaches it.
"""
import os
import shutil
import subprocess
import types

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "symbolic_driver.cpp")
TREE = os.path.join(ROOT, "paper_2309_09061_amd", "csrc", "tree.cpp")

FLAGS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
ENV = {
    "ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    "TSAN_OPTIONS": "halt_on_error=1",
}

CASES = [
    ("1d", 1024, 1, 16, 1.0, "uniform", 1),
    ("ragged", 1000, 2, 24, 1.5, "uniform", 11),
    ("sph", 8192, 3, 64, 2.0, "sphere", 3),
    ("2d_threads", 16384, 2, 16, 1.0, "uniform", 2),
]


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sanitize")
    out = {}
    for name, flags in FLAGS.items():
        exe = str(d / name)
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", *flags, DRIVER, TREE,
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        out[name] = exe
    return out, d


def _read(path):
    raw = np.fromfile(path, dtype=np.int64)
    arrays, p = [], 0
    while p < raw.size:
        n = int(raw[p])
        arrays.append(raw[p + 1:p + 1 + n])
        p += 1 + n
    return arrays


def _product_dict(t, s, ty, tri_ptr, tri):
    tri = tri.reshape(-1, 4)
    kinds = {0: "AA", 1: "AN", 2: "NA", 3: "NN"}
    out = {}
    for b in range(t.size):
        trip = sorted((int(q[0]), kinds[int(q[3])]) for q in tri[tri_ptr[b]:tri_ptr[b + 1]])
        out[(int(t[b]), int(s[b]))] = (int(ty[b]), trip)
    return out


def _oracle_product(ref, bt):
    X = types.SimpleNamespace(V=types.SimpleNamespace(tree=ref), W=types.SimpleNamespace(tree=ref), bt=bt)
    P = O.ProductTree(X, X)
    tmap = {O.SPLIT: 0, O.ADM: 1, O.INADM: 2}
    return {k: (tmap[v], sorted(P.triples[k])) for k, v in P.type.items()}


@pytest.mark.parametrize("build", sorted(FLAGS))
@pytest.mark.parametrize("name,n,dim,leaf,eta,dist,seed", CASES)
def test_symbolic_layer_under_sanitizers(builds, build, name, n, dim, leaf, eta, dist, seed):
    exes, d = builds
    pts = np.ascontiguousarray(W.make_points(seed, n, dim, dist), dtype=np.float64)
    pfile, ofile = str(d / f"{name}_{build}.f64"), str(d / f"{name}_{build}.i64")
    pts.tofile(pfile)
    env = dict(os.environ, **ENV)
    r = subprocess.run([exes[build], pfile, str(n), str(dim), str(leaf), repr(eta), ofile], capture_output=True,
                       text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    perm, off, size, bt_t, bt_s, bt_ty, *prod = _read(ofile)
    ref = O.ClusterTree(pts, leaf)
    bt = O.BlockTree(ref, ref, eta)
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(off, ref.off) and np.array_equal(size, ref.size)
    tmap = {O.SPLIT: 0, O.ADM: 1, O.INADM: 2}
    got = {(int(a), int(b)): int(c) for a, b, c in zip(bt_t, bt_s, bt_ty)}
    assert got == {k: tmap[v] for k, v in bt.type.items()}
    want = _oracle_product(ref, bt)
    for v in range(2):  # X Y, then Y^* X^* (equal here: X = Y with a symmetric block tree)
        t, s, ty, tri_ptr, tri, kind_cnt = prod[6 * v:6 * v + 6]
        assert _product_dict(t, s, ty, tri_ptr, tri) == want
        assert kind_cnt.reshape(-1, 4).sum() == tri.size // 4
