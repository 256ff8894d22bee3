"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every entry point declared in include/h2.h, and
its host-only symbolic work (cluster tree, block tree) equals the oracle's
bit for bit.  Error paths return status codes without touching a device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2309_09061_amd import h2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = h2.load()
    header = open(os.path.join(ROOT, "include", "h2.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(h2_[a-z_0-9]+)\s*\(", header))
    assert len(declared) >= 20
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(h2.EXPORTS) == declared


@pytest.mark.parametrize("name,n,dim,leaf,eta,dist,seed", [
    ("c1", 1024, 1, 16, 1.0, "uniform", 1),
    ("c2", 16384, 2, 64, 1.0, "uniform", 2),
    ("sph", 8192, 3, 64, 2.0, "sphere", 3),
    ("ragged", 1000, 2, 24, 1.5, "uniform", 11),
])
def test_tree_matches_oracle_bit_exact(name, n, dim, leaf, eta, dist, seed):
    pts = W.make_points(seed, n, dim, dist)
    ctx = h2.Context(device=-1)
    T = h2.Tree(ctx, pts, leaf, eta)
    ref = O.ClusterTree(pts, leaf)
    bt = O.BlockTree(ref, ref, eta)
    assert np.array_equal(T.perm, ref.perm)
    off, size, br, bc, btype = T.structure()
    assert np.array_equal(off, ref.off) and np.array_equal(size, ref.size)
    tmap = {O.SPLIT: 0, O.ADM: 1, O.INADM: 2}
    got = {(int(a), int(b)): int(c) for a, b, c in zip(br, bc, btype)}
    assert got == {k: tmap[v] for k, v in bt.type.items()}
    assert T.sizes["depth"] == ref.depth and T.sizes["nclusters"] == ref.nclusters


def test_error_paths_host_only():
    lib = h2.load()
    ctx = h2.Context(device=-1)
    pts = W.make_points(1, 64, 1, "uniform")
    with pytest.raises(h2.H2Error) as e:
        h2.Tree(ctx, pts, 1, 1.0)               # leaf_size < 2
    assert e.value.code == 1
    with pytest.raises(h2.H2Error) as e:
        h2.Tree(ctx, pts, 16, -1.0)             # eta <= 0
    assert e.value.code == 1
    bad = pts.copy()
    bad[3, 0] = np.nan
    with pytest.raises(h2.H2Error) as e:
        h2.Tree(ctx, bad, 16, 1.0)
    assert e.value.code == 7
    with pytest.raises(h2.H2Error) as e:        # empty point set
        h2.Tree(ctx, np.zeros((0, 2)), 16, 1.0)
    assert e.value.code == 1 and "n must be positive" in str(e.value)
    with pytest.raises(h2.H2Error) as e:        # dimension outside 1..3
        h2.Tree(ctx, np.zeros((8, 4)), 16, 1.0)
    assert e.value.code == 1 and "dim" in str(e.value)
    T = h2.Tree(ctx, pts, 16, 1.0)
    with pytest.raises(h2.H2Error) as e:        # device work on a host-only context
        h2.Matrix.kernel(ctx, T, "log", 3)
    assert e.value.code == 1
    out = ctypes.c_void_p()
    assert lib.h2_ctx_create(-2, None, h2.ALLOC_FN(), h2.FREE_FN(), None, ctypes.byref(out)) == 1
    assert lib.h2_tree_sizes(None, None) == 1
    assert "NULL" in lib.h2_last_error().decode()


def test_rank_rule_setting_host_only():
    lib = h2.load()
    ctx = h2.Context(device=-1)
    ctx.set_rank_rule("relF")
    ctx.set_rank_rule("abs")
    assert lib.h2_set_rank_rule(ctx.h, 2) == 1          # unknown rule
    assert lib.h2_set_rank_rule(ctx.h, -1) == 1
    assert lib.h2_set_rank_rule(None, 0) == 1           # NULL context


def test_run_scratch_setting_host_only():
    lib = h2.load()
    ctx = h2.Context(device=-1)
    ctx.set_run_scratch(1 << 20)
    ctx.set_run_scratch(0)                               # back to the default
    ctx.set_run_scratch(-5)
    assert lib.h2_set_run_scratch(None, 1 << 20) == 1    # NULL context


def test_stats_and_export_of_a_tree(tmp_path):
    """h2_stats and h2_export on a tree (host data only)."""
    lib = h2.load()
    ctx = h2.Context(device=-1)
    pts = W.make_points(5, 700, 2, "uniform")
    T = h2.Tree(ctx, pts, 24, 1.5)
    st = h2.stats(T)
    for k in ("n", "dim", "depth", "nclusters", "nblocks", "nadm", "ninadm"):
        assert st[k] == T.sizes[k], k
    assert st["rank_max"] == [0, 0] and st["device_bytes"] == 0
    path = str(tmp_path / "tree.npz")
    h2.export(ctx, T, path)
    d = np.load(path)  # numpy's own reader, no pickles
    off, size, br, bc, bt = T.structure()
    assert int(d["kind"][0]) == 0
    assert np.array_equal(d["perm"], T.perm)
    assert np.array_equal(d["cl_off"], off) and np.array_equal(d["cl_size"], size)
    assert np.array_equal(d["blk_row"], br) and np.array_equal(d["blk_col"], bc)
    assert np.array_equal(d["blk_type"], bt)
    assert np.array_equal(d["points"], pts[T.perm])        # points in cluster order
    # argument errors
    st_c = h2.Stats()
    assert lib.h2_stats(T.h, 7, ctypes.byref(st_c)) == 1
    assert lib.h2_stats(None, 0, ctypes.byref(st_c)) == 1
    assert lib.h2_export(ctx.h, T.h, 0, None) == 1
    assert lib.h2_export(ctx.h, T.h, 0, b"/nonexistent-dir/x.npz") == 1


def test_ctx_create_needs_both_allocator_callbacks():
    lib = h2.load()
    out = ctypes.c_void_p()
    alloc = h2.ALLOC_FN(lambda n, u: None)
    assert lib.h2_ctx_create(-1, None, alloc, h2.FREE_FN(), None, ctypes.byref(out)) == 1
    assert "both allocator callbacks" in lib.h2_last_error().decode()
    assert not out.value
