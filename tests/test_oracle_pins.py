"""Pins of the FP64 oracle against brute force, closed forms and invariants.

Each test fixes one step of the oracle against something other than the
oracle itself: definitions evaluated densely, Gram identities of the
condensation steps, exactness of the method without truncation, scaling
invariance of the block-relative error control and special cases.
"""
import functools
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import h2_oracle as OH
import workloads as W
from oracle_cases import dense, problem, product, rel2, relF

CASES = ["1d", "2d", "2d64", "sph"]


# --------------------------------------------------------------------------
# P1: cluster tree and block tree (Definitions "Cluster tree", "Block tree"; R1-R3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", CASES)
def test_cluster_tree_definition(name):
    pts, tree, bt, _, _ = problem(name)
    n, leaf = tree.n, {"1d": 16, "2d": 32, "2d64": 64, "sph": 32}[name]
    assert sorted(tree.perm.tolist()) == list(range(n))
    assert tree.size[0] == n and tree.off[0] == 0
    for c in range(tree.nclusters):
        idx = set(tree.perm[tree.rng(c)].tolist())
        sub = pts[list(idx)]
        # tight boxes
        assert np.array_equal(tree.bmin[c], sub.min(axis=0))
        assert np.array_equal(tree.bmax[c], sub.max(axis=0))
        kids = tree.children[c]
        if kids:
            assert len(kids) == 2
            parts = [set(tree.perm[tree.rng(k)].tolist()) for k in kids]
            assert parts[0] | parts[1] == idx and not (parts[0] & parts[1])
            assert len(parts[0]) == len(idx) // 2
            # median split along the longest edge, (coordinate, index) order
            ax = int(np.argmax(tree.bmax[c] - tree.bmin[c]))
            key = lambda i: (pts[i, ax], i)
            assert max(map(key, parts[0])) < min(map(key, parts[1]))
        else:
            assert tree.size[c] <= leaf and tree.level[c] == tree.depth


@pytest.mark.parametrize("name", CASES)
def test_block_tree_partition_and_admissibility(name):
    pts, tree, bt, _, _ = problem(name)
    n = tree.n
    cover = np.zeros((n, n), dtype=np.int32)
    for (t, s), ty in bt.type.items():
        if ty == O.SPLIT:
            continue
        cover[tree.rng(t), tree.rng(s)] += 1
        P, Qp = pts[tree.perm[tree.rng(t)]], pts[tree.perm[tree.rng(s)]]
        diam_t = np.linalg.norm(P.max(0) - P.min(0))
        diam_s = np.linalg.norm(Qp.max(0) - Qp.min(0))
        gap = np.maximum(0, np.maximum(Qp.min(0) - P.max(0), P.min(0) - Qp.max(0)))
        dist = np.linalg.norm(gap)
        adm = dist > 0 and max(diam_t, diam_s) <= bt.eta * dist
        assert adm == (ty == O.ADM)
        if ty == O.INADM:
            assert tree.is_leaf(t) and tree.is_leaf(s)
    assert np.all(cover == 1)
    # every non-leaf block is inadmissible and has chil(t) x chil(s) as children
    for (t, s), ty in bt.type.items():
        if ty == O.SPLIT:
            assert not bt.admissible(t, s)
            assert sorted(bt.children[(t, s)]) == sorted(itertools.product(tree.children[t], tree.children[s]))


# --------------------------------------------------------------------------
# P2: Chebyshev H^2 construction (Example "Integral operator"; R4, R5)
# --------------------------------------------------------------------------
def test_lagrange_cardinality():
    nodes = O.cheb_nodes(-0.3, 1.7, 5)
    assert np.allclose(O.lagrange(nodes, nodes), np.eye(5), atol=1e-14)
    # nodes are the roots of T_5 mapped to [-0.3, 1.7]
    u = (nodes - 0.7) / 1.0
    assert np.allclose(np.cos(5 * np.arccos(u)), 0, atol=1e-13)


@pytest.mark.parametrize("name", CASES)
def test_cluster_basis_nested(name):
    _, tree, _, X, _ = problem(name)
    Vf = X.V.full()
    m = {"1d": 4, "2d": 3, "2d64": 4, "sph": 3}[name]
    for c in range(1, tree.nclusters):
        p = tree.parent[c]
        direct = OH._tensor_lagrange(tree, p, m, tree.points[tree.rng(c)])   # V_parent restricted to c
        assert np.abs(Vf[c] @ X.V.transfer[c] - direct).max() <= 1e-12 * max(1.0, np.abs(direct).max())


@pytest.mark.parametrize("dim,order", [(1, 3), (2, 3), (3, 3)])
def test_polynomial_kernel_reproduced_exactly(dim, order):
    pts = W.make_points(5, 300, dim, "uniform")
    tree = O.ClusterTree(pts, 16)
    bt = O.BlockTree(tree, tree, 1.0)
    X = O.kernel_h2(tree, bt, "poly2", order)
    exact = (tree.points @ tree.points.T) ** 2
    assert relF(X.dense(), exact) < 1e-12


@pytest.mark.parametrize("name", CASES)
def test_matvec_equals_dense(name):
    _, tree, _, X, Y = problem(name)
    Xd, Yd, _ = dense(name)
    x = W.probe_vectors(3, tree.n, 3)
    assert relF(X.matvec(x), Xd @ x) < 1e-13
    assert relF(Y.matvec(x), Yd @ x) < 1e-13
    assert relF(X.transposed().matvec(x), Xd.T @ x) < 1e-13


def test_kernel_entries_and_diagonal():
    _, tree, _, X, Y = problem("2d")
    Xd, Yd, _ = dense("2d")
    p = tree.points
    i, j = 5, 300
    # a nearfield entry is the kernel itself; the diagonal follows R5
    r = np.linalg.norm(p[i] - p[j])
    for b, N in X.N.items():
        t, s = b
        if tree.off[t] <= i < tree.off[t] + tree.size[t] and tree.off[s] <= j < tree.off[s] + tree.size[s]:
            assert np.isclose(Xd[i, j], np.log(r), rtol=1e-14)
            assert np.isclose(Yd[i, j], np.exp(-r), rtol=1e-14)
    assert np.all(np.diag(Xd) == 0.0) and np.all(np.diag(Yd) == 1.0)


def _raw_kernel(kind, pts):
    """The kernel matrix written from its definition on the raw points in
    input order (Section 7, single-layer kernel 1/(4 pi |x-y|); 1/|x-y| of the
    volume workload), zero diagonal (R5)."""
    d = pts[:, None, :] - pts[None, :, :]
    r = np.sqrt((d * d).sum(axis=-1))
    with np.errstate(divide="ignore"):
        K = 1.0 / r if kind == "inv" else 1.0 / (4.0 * np.pi * r)
    np.fill_diagonal(K, 0.0)
    return K


@pytest.mark.parametrize("kind,dist,seed", [("inv4pi", "sphere", 3), ("inv", "uniform", 5)])
def test_singular_kernel_entries_from_raw_points(kind, dist, seed):
    """The singular kernels of the sphere and cube workloads against the raw
    kernel matrix: nearfield entries exactly, the interpolated far field
    within the interpolation error, which shrinks with the order (so a wrong
    constant, power or diagonal in the oracle's kernel fails here)."""
    pts = W.make_points(seed, 512, 3, dist)
    tree = O.ClusterTree(pts, 32)
    bt = O.BlockTree(tree, tree, 2.0)
    Kc = _raw_kernel(kind, pts)[np.ix_(tree.perm, tree.perm)]
    errs = []
    for order in (3, 5):
        X = O.kernel_h2(tree, bt, kind, order)
        Xd = X.dense()
        for (t, s) in X.N:
            blk = Kc[tree.rng(t), tree.rng(s)]
            assert np.array_equal(Xd[tree.rng(t), tree.rng(s)], blk)
        assert np.all(np.diag(Xd) == 0.0)
        for (t, s) in X.S:
            blk = Kc[tree.rng(t), tree.rng(s)]
            assert np.abs(Xd[tree.rng(t), tree.rng(s)] - blk).max() <= 0.1 * np.abs(blk).max()
        errs.append(relF(Xd, Kc))
    assert errs[0] < 2e-3
    assert errs[1] < errs[0] / 5


# --------------------------------------------------------------------------
# P3-P5: set-up quantities (basis weights, basis products, total weights)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", CASES)
def test_basis_weights_gram(name):
    _, tree, _, _, Y = problem(name)
    R = O.basis_weights(Y.W)
    Wf = Y.W.full()
    for r in range(tree.nclusters):
        G = Wf[r].T @ Wf[r]
        assert R[r].shape[0] == min(Y.W.rank[r], tree.size[r])
        assert np.abs(R[r].T @ R[r] - G).max() <= 1e-13 * np.abs(G).max()


@pytest.mark.parametrize("name", CASES)
def test_cluster_basis_products_dense(name):
    _, tree, _, X, Y = problem(name)
    P = O.cluster_basis_products(X.W, Y.V)
    Wf, Vf = X.W.full(), Y.V.full()
    for s in range(tree.nclusters):
        D = Wf[s].T @ Vf[s]
        assert np.abs(P[s] - D).max() <= 1e-13 * np.abs(D).max()


@pytest.mark.parametrize("name", CASES)
def test_total_weights_gram(name):
    """V_{Y,s} Z_s^* Z_s V_{Y,s}^* equals the Gram matrix of the scaled dense
    rows Y|_{s x r} of every admissible block (s*, r) with s* an ancestor of
    s or s itself; the scale is 1/||S_{Y,s*r} W_{Y,r}^*||_2 (Section 5)."""
    _, tree, _, _, Y = problem(name)
    _, Yd, _ = dense(name)
    Z = O.total_weights(Y, O.basis_weights(Y.W))
    Vf, Wf = Y.V.full(), Y.W.full()
    for s in range(tree.nclusters):
        lhs = Vf[s] @ Z[s].T @ Z[s] @ Vf[s].T
        rhs = np.zeros_like(lhs)
        anc = s
        while anc >= 0:
            for (a, r), ty in Y.bt.type.items():
                if a == anc and ty == O.ADM:
                    w = np.linalg.norm(Y.S[(a, r)] @ Wf[r].T, 2)
                    B = Yd[tree.rng(s), tree.rng(r)] / w
                    rhs += B @ B.T
            anc = tree.parent[anc]
        assert np.abs(lhs - rhs).max() <= 1e-12 * max(np.abs(rhs).max(), 1e-300)


# --------------------------------------------------------------------------
# P6: phase 1 (Section 4, Figure "induced_basis"; Section 5)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_phase1_basis_isometric_and_keeps_VX(name, eps):
    _, tree, _, X, _ = problem(name)
    p1, _ = product(name, eps)
    for side, VX in ((p1.row, X.V.full()), (p1.col, problem(name)[4].W.full())):
        Qf = side.Q.full()
        for t in range(tree.nclusters):
            Q = Qf[t]
            assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
            res = VX[t] - Q @ (Q.T @ VX[t])
            # the numerical range (relative tolerance 1e-12) is kept exactly
            assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(VX[t])


@pytest.mark.parametrize("name", ["1d", "2d", "2d64"])
@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_phase1_kept_range_is_thin_householder_factor(name, eps):
    """Where V_{X,t} has full numerical rank (the 1-D and 2-D cases), the
    kept part of Q_t reduces to the paper's literal construction (Section 4,
    leaf case): k1 = min(k, rows of V_{X,t}) on every cluster, and the first
    k1 columns of Q_t span the range of the thin Householder factor of
    V_{X,t} (the 2-D and 1-D inputs have no numerical rank deficiency)."""
    _, tree, _, X, _ = problem(name)
    p1, _ = product(name, eps)
    k = X.V.rank[0]
    for side in (p1.row, p1.col):
        for t in range(tree.nclusters):
            VX = side.assembled[t][0]
            k1 = side.RX[t].shape[0]
            assert k1 == min(k, VX.shape[0]), (t, k1, VX.shape)
            if tree.is_leaf(t):
                Qt = side.Q.leaf[t]
            else:
                Qt = np.vstack([side.Q.transfer[ch] for ch in tree.children[t]])
            Qh, _ = np.linalg.qr(VX)               # thin Householder factor
            P1 = Qt[:, :k1] @ Qt[:, :k1].T
            assert np.abs(P1 - Qh @ Qh.T).max() < 1e-12


@pytest.mark.parametrize("name", CASES)
def test_phase1_condensation_gram(name):
    """The assembled remainder of induced_basis(t) has the Gram matrix of the
    uncondensed block-scaled products X|_{t x s} Y|_{s x r} (leaf), projected
    onto the children's bases (non-leaf)."""
    _, tree, _, X, Y = problem(name)
    Xd, Yd, _ = dense(name)
    p1, _ = product(name, 1e-6)
    Qf = p1.row.Q.full()
    Vyf, Wyf = Y.V.full(), Y.W.full()
    for t in range(tree.nclusters):
        if tree.is_leaf(t):
            U = np.eye(tree.size[t])
        else:
            U = np.zeros((tree.size[t], sum(p1.row.Q.rank[c] for c in tree.children[t])))
            o = 0
            for c in tree.children[t]:
                sl = slice(tree.off[c] - tree.off[t], tree.off[c] - tree.off[t] + tree.size[c])
                U[sl, o:o + p1.row.Q.rank[c]] = Qf[c]
                o += p1.row.Q.rank[c]
        B = []
        for (a, s), ty in X.bt.type.items():
            if a != t or ty == O.ADM:
                continue
            XV = U.T @ Xd[tree.rng(t), tree.rng(s)] @ Vyf[s]
            ws = np.linalg.norm(XV, 2)
            if ws == 0:
                continue
            anc = s
            while anc >= 0:
                for (b0, r), tyy in Y.bt.type.items():
                    if b0 == anc and tyy == O.ADM:
                        wr = np.linalg.norm(Y.S[(b0, r)] @ Wyf[r].T, 2)
                        B.append(U.T @ Xd[tree.rng(t), tree.rng(s)] @ Yd[tree.rng(s), tree.rng(r)] / (ws * wr))
                anc = tree.parent[anc]
        VX, Vrest = p1.row.assembled[t]
        assert np.abs(VX - U.T @ X.V.full()[t]).max() <= 1e-12 * np.abs(VX).max()
        if not B:
            assert Vrest.shape[1] == 0 or np.abs(Vrest).max() == 0
            continue
        Bm = np.hstack(B)
        lhs, rhs = Vrest @ Vrest.T, Bm @ Bm.T
        assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()


@pytest.mark.parametrize("name", CASES)
def test_phase1_exact_without_truncation(name):
    """eps = 0: G represents X Y exactly (Section 3, exact induced representation)."""
    _, _, XY = dense(name)
    p1, _ = product(name, 0.0)
    assert relF(p1.G.dense(), XY) < 1e-12


def test_rank_rule_strict():
    assert O.choose_rank(np.array([3.0, 1e-6, 1e-6 * (1 - 1e-15), 0.0]), 1e-6) == 1
    assert O.choose_rank(np.array([]), 1e-3) == 0


# --------------------------------------------------------------------------
# P7: product block tree and the intermediate product (R13, R14)
# --------------------------------------------------------------------------
def _brute_triples(X, Y):
    tree = X.V.tree
    reached = {}
    for lev in range(tree.depth + 1):
        cl = list(tree.clusters_at(lev))
        for t, s, r in itertools.product(cl, cl, cl):
            if (t, s) not in X.bt.type or (s, r) not in Y.bt.type:
                continue
            if lev > 0:
                pt, ps, pr = tree.parent[t], tree.parent[s], tree.parent[r]
                if not (X.bt.type.get((pt, ps)) == O.SPLIT and Y.bt.type.get((ps, pr)) == O.SPLIT):
                    continue
            reached.setdefault((t, r), []).append(s)
    return reached


@pytest.mark.parametrize("name", ["1d", "2d"])
def test_product_tree_brute_force(name):
    _, tree, _, X, Y = problem(name)
    PT = O.ProductTree(X, Y)
    reached = _brute_triples(X, Y)
    assert set(reached) == set(PT.type)
    for b, mids in reached.items():
        kinds = [(X.bt.type[(b[0], s)], Y.bt.type[(s, b[1])]) for s in mids]
        if any(a == O.SPLIT and c == O.SPLIT for a, c in kinds):
            want = O.SPLIT
        elif any(a == O.INADM and c == O.INADM for a, c in kinds):
            want = O.INADM
        else:
            want = O.ADM
        assert PT.type[b] == want
        assert sorted(PT.split[b] + [s for s, _ in PT.triples[b]]) == sorted(mids)


@pytest.mark.parametrize("name", ["1d", "2d", "sph"])
def test_intermediate_product_dense_definition(name):
    """At eps > 0, G equals sum over terminated triples of
    P_row X|_{ts} Y|_{sr} P_col evaluated densely (R14)."""
    _, tree, _, X, Y = problem(name)
    Xd, Yd, _ = dense(name)
    p1, _ = product(name, 1e-4)
    Qf, QWf = p1.row.Q.full(), p1.col.Q.full()
    reached = _brute_triples(X, Y)
    Gdef = np.zeros_like(Xd)
    for (t, r), mids in reached.items():
        for s in mids:
            tx, ty = X.bt.type[(t, s)], Y.bt.type[(s, r)]
            if tx == O.SPLIT and ty == O.SPLIT:
                continue
            M = Xd[tree.rng(t), tree.rng(s)] @ Yd[tree.rng(s), tree.rng(r)]
            if not (tx == O.INADM and ty == O.INADM):
                if tx != O.ADM:
                    M = Qf[t] @ (Qf[t].T @ M)
                if ty != O.ADM:
                    M = (M @ QWf[r]) @ QWf[r].T
            Gdef[tree.rng(t), tree.rng(r)] += M
    assert relF(p1.G.dense(), Gdef) < 1e-12


# --------------------------------------------------------------------------
# P8: phase 2 (Section 6, Figures "match_column" and "basis"; R10-R12, R15)
# --------------------------------------------------------------------------
def _tik_rows(TIK, tree):
    out = {}
    for (t, r), ty in TIK.type.items():
        if ty == O.ADM:
            out.setdefault(t, []).append(r)
    return out


@pytest.mark.parametrize("name", CASES)
def test_phase2_condensation_gram(name):
    """C_t (leaf) and Chat_t (non-leaf) carry the Gram matrix of the block-
    scaled dense G_t = G|_{t x R_t} (projected onto the children's new
    bases), with omega_b = 1/||G|_b||_F (R10)."""
    _, tree, bt, _, _ = problem(name)
    p1, p2 = product(name, 1e-6)
    Gd = p1.G.dense()
    QZ = p2.row.Q.full()
    rows = _tik_rows(bt, tree)
    for t in range(tree.nclusters):
        if tree.is_leaf(t):
            U = np.eye(tree.size[t])
        else:
            U = np.zeros((tree.size[t], sum(p2.row.Q.rank[c] for c in tree.children[t])))
            o = 0
            for c in tree.children[t]:
                sl = slice(tree.off[c] - tree.off[t], tree.off[c] - tree.off[t] + tree.size[c])
                U[sl, o:o + p2.row.Q.rank[c]] = QZ[c]
                o += p2.row.Q.rank[c]
        B = []
        anc = t
        while anc >= 0:
            for r in rows.get(anc, []):
                blk = Gd[tree.rng(anc), tree.rng(r)]
                nb = np.linalg.norm(blk)
                assert np.isclose(p2.row.omega.get((anc, r), 0.0) * nb, 1.0 if nb > 0 else 0.0, rtol=1e-12)
                if nb > 0:
                    B.append(U.T @ Gd[tree.rng(t), tree.rng(r)] / nb)
            anc = tree.parent[anc]
        C = p2.row.C[t]
        if not B:
            assert C.size == 0 or np.abs(C).max() < 1e-300
            continue
        Bm = np.hstack(B)
        assert np.abs(C @ C.T - Bm @ Bm.T).max() <= 1e-11 * np.abs(Bm @ Bm.T).max()


@pytest.mark.parametrize("name", CASES)
def test_phase2_bases_isometric(name):
    _, tree, _, _, _ = problem(name)
    _, p2 = product(name, 1e-6)
    for side in (p2.row, p2.col):
        Qf = side.Q.full()
        for t in range(tree.nclusters):
            if Qf[t].shape[1]:        # the root has no admissible block and may have rank 0
                assert np.abs(Qf[t].T @ Qf[t] - np.eye(Qf[t].shape[1])).max() < 1e-13


@pytest.mark.parametrize("name", ["1d", "2d", "sph"])
def test_final_product_dense_definition(name):
    """Z equals the dense evaluation of R15 from the densified bases."""
    _, tree, bt, _, _ = problem(name)
    p1, p2 = product(name, 1e-4)
    Gd = p1.G.dense()
    QZ, QZW = p2.row.Q.full(), p2.col.Q.full()
    Zdef = np.zeros_like(Gd)
    for (t, r), ty in bt.type.items():
        blk = Gd[tree.rng(t), tree.rng(r)]
        if ty == O.ADM:
            Zdef[tree.rng(t), tree.rng(r)] = QZ[t] @ (QZ[t].T @ blk @ QZW[r]) @ QZW[r].T
        elif ty == O.INADM:
            Zdef[tree.rng(t), tree.rng(r)] = blk
    assert relF(p2.Z.dense(), Zdef) < 1e-12


@pytest.mark.parametrize("name", CASES)
def test_final_exact_without_truncation(name):
    """eps = 0 in both phases: Z = G = X Y."""
    _, _, XY = dense(name)
    _, p2 = product(name, 0.0)
    assert relF(p2.Z.dense(), XY) < 1e-12


# --------------------------------------------------------------------------
# P9: error bound (Section 5; Tables "slp", "dlp": errors stay below eps)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_final_error_below_eps(name, eps):
    _, _, XY = dense(name)
    p1, p2 = product(name, eps)
    e1, e2 = rel2(p1.G.dense(), XY), rel2(p2.Z.dense(), XY)
    assert e1 <= eps and e2 <= eps
    # truncation actually happened (ranks below the untruncated ones)
    _, p20 = product(name, 0.0)
    assert sum(p2.row.Q.rank.values()) < sum(p20.row.Q.rank.values())


# --------------------------------------------------------------------------
# P10: special cases
# --------------------------------------------------------------------------
def test_identity_factor():
    pts, tree, bt, _, Y = problem("2d")
    I = O.identity_h2(tree, bt, 3)
    _, Yd, _ = dense("2d")
    _, p2 = O.multiply(I, Y, bt, 1e-6)
    assert rel2(p2.Z.dense(), Yd) <= 1e-6


def test_zero_factor():
    _, tree, bt, X, Y = problem("2d")
    _, p2 = O.multiply(O.scaled(X, 0.0), Y, bt, 1e-6)
    assert np.abs(p2.Z.dense()).max() == 0.0


@pytest.mark.parametrize("alpha", [1e-3, 7.5e4])
def test_scaling_invariance_of_error_control(alpha):
    """Block-relative error control (Section 5, R8-R10): scaling X scales Z
    and leaves every rank unchanged."""
    _, tree, bt, X, Y = problem("2d")
    p1, p2 = product("2d", 1e-6)
    q1, q2 = O.multiply(O.scaled(X, alpha), Y, bt, 1e-6)
    assert q1.row.Q.rank == p1.row.Q.rank and q1.col.Q.rank == p1.col.Q.rank
    assert q2.row.Q.rank == p2.row.Q.rank and q2.col.Q.rank == p2.col.Q.rank
    assert relF(q2.Z.dense(), alpha * p2.Z.dense()) < 1e-11


def test_low_rank_kernel_ranks():
    """(x.y)^2 in 2-D has rank d(d+1)/2 = 3 and is reproduced exactly by
    order-3 interpolation: above roundoff, phase 1 adds nothing to range(V_X)
    (k2 = 0) and phase 2 finds rank 3 (rank 0 for coarse clusters without
    any admissible block at or above them); Z is then exact.  At eps = 1e-4 block-relative
    truncation may drop a weak direction, within the eps bound."""
    pts = W.make_points(9, 400, 2, "uniform")
    tree, bt, X, Y = O.build_problem(pts, 25, 1.0, 3, "poly2", "poly2")
    XY = X.dense() @ Y.dense()
    p1, p2 = O.multiply(X, Y, bt, 1e-10)
    assert set(p1.row.Q.rank.values()) == {9} and set(p1.col.Q.rank.values()) == {9}
    has_adm = {t for (t, r), ty in bt.type.items() if ty == O.ADM}
    for c in range(tree.nclusters):
        a, row_star = c, False
        while a >= 0:
            row_star |= a in has_adm
            a = tree.parent[a]
        assert p2.row.Q.rank[c] == (3 if row_star else 0)
    assert rel2(p2.Z.dense(), XY) < 1e-13
    _, q2 = O.multiply(X, Y, bt, 1e-4)
    assert max(q2.row.Q.rank.values()) <= 3 and rel2(q2.Z.dense(), XY) <= 1e-4


def test_symmetric_product_bases_coincide():
    """X = Y symmetric: the column pass sees the same data as the row pass."""
    p1, p2 = product("1d", 1e-6)
    assert p1.row.Q.rank == p1.col.Q.rank
    assert p2.row.Q.rank == p2.col.Q.rank


# --------------------------------------------------------------------------
# R21 (variant of R9): relative-Frobenius truncation
# --------------------------------------------------------------------------
def test_rel_frobenius_rank_rule_brute_force():
    """The rank is the smallest k whose discarded tail has Frobenius norm at
    most eps times that of all singular values (brute force over k)."""
    rng = np.random.default_rng(21)
    for _ in range(300):
        n = int(rng.integers(0, 9))
        sig = np.sort(rng.random(n) * 10.0 ** rng.integers(-4, 3, n))[::-1]
        eps = 10.0 ** rng.uniform(-5, 0)
        total = np.sqrt(np.sum(sig ** 2))
        ok = [k for k in range(n + 1) if np.sqrt(np.sum(sig[k:] ** 2)) <= eps * total]
        assert O.choose_rank(sig, eps, O.RANK_REL_FROB) == min(ok)
    assert O.choose_rank(np.zeros(3), 0.1, O.RANK_REL_FROB) == 0
    assert O.choose_rank(np.array([4.0, 3.0]), 0.6, O.RANK_REL_FROB) == 1  # tail 3 = 0.6 * 5: discarded


def _stacked_transfers(Q, tree, t):
    return np.vstack([Q.transfer[ch] for ch in tree.children[t]])


@pytest.mark.parametrize("name", ["1d", "2d"])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_rel_frobenius_truncation_of_each_cluster(name, eps):
    """Phase 2 under R21: each condensed matrix C_t (Chat_t) keeps all but at
    most eps of its Frobenius norm in the span of the new basis, checked from
    the matrices themselves (projection residual), and phase 1's remainder
    likewise after the kept range of V_X."""
    _, tree, bt, X, Y = problem(name)
    p1, p2 = O.multiply(X, Y, bt, eps, rule=O.RANK_REL_FROB)
    for side in (p2.row, p2.col):
        for t, C in side.C.items():
            if C.size == 0:
                continue
            Q = side.Q.leaf[t] if tree.is_leaf(t) else (
                _stacked_transfers(side.Q, tree, t) if side.Q.rank[t] else np.zeros((C.shape[0], 0)))
            res = C - Q @ (Q.T @ C)
            assert np.linalg.norm(res) <= eps * np.linalg.norm(C) * (1 + 1e-10) + 1e-14 * np.linalg.norm(C)
    Qf = p1.row.Q.full()
    for t, (VX, Vrest) in p1.row.assembled.items():
        if Vrest.size == 0:
            continue
        Q = Qf[t] if tree.is_leaf(t) else _stacked_transfers(p1.row.Q, tree, t)
        Ux, sx, _ = np.linalg.svd(VX, full_matrices=True)
        k1 = int(np.count_nonzero(sx > OH.VX_RTOL * sx[0])) if sx.size and sx[0] > 0 else 0
        rem = Vrest - Ux[:, :k1] @ (Ux[:, :k1].T @ Vrest)       # remainder outside range V_X
        res = Vrest - Q @ (Q.T @ Vrest)
        assert np.linalg.norm(res) <= eps * np.linalg.norm(rem) * (1 + 1e-10) + 1e-13 * np.linalg.norm(Vrest)


@pytest.mark.parametrize("name", ["1d", "2d"])
def test_rel_frobenius_exact_without_truncation(name):
    _, _, bt, X, Y = problem(name)
    _, _, XY = dense(name)
    p1, p2 = O.multiply(X, Y, bt, 0.0, rule=O.RANK_REL_FROB)
    assert relF(p1.G.dense(), XY) < 1e-12
    assert relF(p2.Z.dense(), XY) < 1e-12


# --------------------------------------------------------------------------
# P11: the work ledger (algorithmic flop counts per step) against the
# method's linear complexity (Section 6, closing complexity estimate; the
# bounded run time per degree of freedom of Section 7) and against a
# brute-force count of its dominant term
# --------------------------------------------------------------------------
def _ledger_of(n, dim, leaf, order, kx, ky, eps, seed, eta=1.0):
    pts = W.make_points(seed, n, dim, "uniform")
    tree, bt, X, Y = O.build_problem(pts, leaf, eta, order, kx, ky)
    with O.counting() as led:
        O.multiply(X, Y, bt, eps)
    return tree, bt, led


def test_work_ledger_linear_complexity_1d():
    """Work per degree of freedom stays bounded as n grows (O(n k^2) total)."""
    per = []
    for n in (1024, 2048, 4096, 8192, 16384):
        _, _, led = _ledger_of(n, 1, 16, 4, "log", "log", 1e-8, 1)
        per.append(sum(led.values()) / n)
    assert max(per) / min(per) < 1.15, per
    assert max(per[2:]) / min(per[2:]) < 1.03, per


def test_work_ledger_steps_and_dense_triples():
    """Every step is counted, and the G formation's products include the
    dense nearfield-times-nearfield products 2 #t #s #r of every leaf triple
    (t, s, r) whose two factor blocks are inadmissible leaves (enumerated by
    brute force from the block tree), plus at most the small coupling
    products of the remaining triples and blocks."""
    tree, bt, led = _ledger_of(1024, 2, 32, 3, "log", "expneg", 1e-6, 2)
    steps = {s for s, _ in led}
    assert {"setup", "p1_row", "p1_col", "p1_mat", "p2_row", "p2_col", "p2_mat"} <= steps
    for st in ("p1_row", "p1_col", "p2_row", "p2_col"):
        assert led[(st, "svd")] > 0 and led[(st, "qr")] > 0 and led[(st, "gemm")] > 0
    inad = [(t, s) for (t, s), ty in bt.type.items() if ty == O.INADM]
    by_row = {}
    for t, s in inad:
        by_row.setdefault(t, []).append(s)
    dense = 0.0
    for t, s in inad:
        for r in by_row.get(s, []):
            dense += 2.0 * tree.size[t] * tree.size[s] * tree.size[r]
    k = 9
    nblocks = len(bt.type)
    small = 2.0 * (2 * k) ** 3 * 5 * (nblocks ** 2)   # generous bound on the rest
    assert dense <= led[("p1_mat", "gemm")] <= dense + small


# --------------------------------------------------------------------------
# The double-layer kernel of Section 7 (<n(x), x - y> / (4 pi |x - y|^3) on
# the surface of [-1, 1]^3): derivative interpolation basis, raw entries,
# convergence, and the product of a non-symmetric matrix with itself
# --------------------------------------------------------------------------
def test_lagrange_derivative_reproduces_polynomial_derivatives():
    rng = np.random.default_rng(5)
    for m in (2, 3, 4, 5):
        a, b = sorted(rng.uniform(-3, 3, 2))
        nodes = OH.cheb_nodes(a, b, m)
        x = np.concatenate([rng.uniform(a - 1, b + 1, 40), nodes])   # nodes included
        coef = rng.standard_normal(m)                                 # degree m - 1
        p = np.polynomial.polynomial.polyval(nodes, coef)
        dp = np.polynomial.polynomial.polyval(x, np.polynomial.polynomial.polyder(coef))
        got = OH.lagrange_derivative(nodes, x) @ p
        assert np.abs(got - dp).max() <= 1e-11 * max(1.0, np.abs(dp).max())


@functools.lru_cache(maxsize=None)
def _dlp_problem(n=1536, order=3, leaf=32, seed=6):
    pts = W.make_points(seed, n, 3, "cube_surface")
    nrm = W.cube_surface_normals(pts)
    tree, bt, X, _ = O.build_problem(pts, leaf, 2.0, order, "dlp", "dlp", normals=nrm)
    return pts, nrm, tree, bt, X


def test_cube_surface_points_and_normals():
    pts = W.make_points(6, 3000, 3, "cube_surface")
    nrm = W.cube_surface_normals(pts)
    assert np.all(np.abs(pts) <= 1.0) and np.allclose(np.max(np.abs(pts), axis=1), 1.0, rtol=0, atol=0)
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
    # each normal is the outward axis of the face the point lies on
    assert np.all(np.sum(nrm * pts, axis=1) == 1.0)


def test_dlp_entries_from_raw_points():
    """Nearfield entries equal <n(x_i), x_i - x_j>/(4 pi |x_i - x_j|^3) from the
    raw points and normals (0 on the diagonal and, exactly, for two points of
    the same face); the far field converges as the order grows."""
    pts, nrm, tree, bt, X = _dlp_problem()
    Xd = X.dense()
    P, Nr = pts[tree.perm], nrm[tree.perm]
    raw = np.zeros_like(Xd)
    for i in range(tree.n):
        d = P[i] - P
        r = np.linalg.norm(d, axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            raw[i] = (d @ Nr[i]) / (4.0 * np.pi * r ** 3)
        raw[i, i] = 0.0
    near = np.zeros(Xd.shape, dtype=bool)
    for (t, s), ty in bt.type.items():
        if ty == O.INADM:
            near[tree.rng(t), tree.rng(s)] = True
    assert np.abs(Xd[near] - raw[near]).max() <= 1e-15 * np.abs(raw[near]).max()
    same_face = (Nr @ Nr.T) == 1.0
    assert np.all(Xd[near & same_face] == 0.0)
    errs = []
    for order in (2, 3, 4):
        Xo = _dlp_problem(order=order)[4].dense()
        errs.append(np.linalg.norm((Xo - raw)[~near]) / np.linalg.norm(raw[~near]))
    # interpolation error of the far field falls by more than 2 per order
    assert errs[0] > 2 * errs[1] and errs[1] > 2 * errs[2], errs


def test_dlp_row_basis_nested():
    """The normal-derivative row basis is nested: expanding the transfers
    gives the derivative basis of the parent evaluated on the child's points."""
    pts, nrm, tree, bt, X = _dlp_problem(n=600, leaf=16)
    Vf = X.V.full()
    Nr = nrm[tree.perm]
    for c in range(1, tree.nclusters):
        if tree.is_leaf(c):
            continue
        r = tree.rng(c)
        direct = OH._tensor_normal_derivative(tree, c, 3, tree.points[r], Nr[r], OH._cube_boxes)
        assert np.abs(Vf[c] - direct).max() <= 1e-11 * np.abs(direct).max()


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_dlp_product_error_and_adjoint_passes(eps):
    """X X for the non-symmetric double-layer matrix: exact without
    truncation, within eps otherwise; the column pass of X Y equals the row
    pass of Y^* X^* (same ranks), and row and column ranks differ."""
    pts, nrm, tree, bt, X = _dlp_problem()
    Xd = X.dense()
    XY = Xd @ Xd
    p1, p2 = O.multiply(X, X, bt, eps)
    Zd = p2.Z.dense()
    if eps == 0.0:
        assert relF(p1.G.dense(), XY) <= 1e-12 and relF(Zd, XY) <= 1e-12
        return
    assert rel2(Zd, XY) <= eps
    Xt = X.transposed()
    q1 = O.Phase1(Xt, Xt, eps)
    nc = tree.nclusters
    assert [p1.col.Q.rank[c] for c in range(nc)] == [q1.row.Q.rank[c] for c in range(nc)]
    assert [p1.row.Q.rank[c] for c in range(nc)] != [p1.col.Q.rank[c] for c in range(nc)]


def test_block_scaling_ignores_rounding_level_blocks():
    """Section 5 scaling with reading R8: blocks of the double-layer product
    that vanish in exact arithmetic (two clusters on one face) come out of
    the interpolated couplings at the rounding level; scaled to unit norm
    they would decide ranks by rounding noise.  Dropping blocks at most
    BLOCK_RTOL of their level's largest makes the rank profiles invariant
    under a perturbation of X at 1e-14; without the rule they are not."""
    pts, nrm, tree, bt, X = _dlp_problem()
    rng = np.random.default_rng(1)
    Xp = O.H2Matrix(X.V, X.W, X.bt, {b: m * (1 + 1e-14 * rng.standard_normal(m.shape)) for b, m in X.S.items()},
                    {b: m * (1 + 1e-14 * rng.standard_normal(m.shape)) for b, m in X.N.items()})

    def moved():
        a, b = O.Phase1(X, X, 1e-4), O.Phase1(Xp, Xp, 1e-4)
        return sum(a.row.Q.rank[c] != b.row.Q.rank[c] or a.col.Q.rank[c] != b.col.Q.rank[c]
                   for c in range(tree.nclusters))
    assert moved() == 0
    saved = OH.BLOCK_RTOL
    try:
        OH.BLOCK_RTOL = 0.0
        assert moved() > 0
    finally:
        OH.BLOCK_RTOL = saved


# --------------------------------------------------------------------------
# Z <- Z + X Y with Z != 0 (the operation of the Introduction; reading R16:
# the old Z's bases are kept exactly, as phase 1 keeps range(V_X))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name,eps", [("2d", 0.0), ("2d", 1e-6), ("sph", 1e-4), ("1d", 1e-8)])
def test_update_of_nonzero_target(name, eps):
    """Z1 = X Y, then Z2 = Z1 + X Y and Z3 = Y + X Y (a kernel matrix with
    non-isometric bases as the old Z): exact at eps = 0, else within eps of
    the exact sums; the old Z's row and column bases stay inside the new
    ones at every cluster."""
    _, tree, bt, X, Y = problem(name)
    Xd, Yd, XY = dense(name)
    _, p2a = O.multiply(X, Y, bt, eps)
    for old, old_dense in ((p2a.Z, p2a.Z.dense()), (Y, Yd)):
        _, p2 = O.multiply(X, Y, bt, eps, Zold=old)
        err = rel2(p2.Z.dense() - old_dense, XY)
        assert err <= (1e-12 if eps == 0 else eps), err
        for new, kept in ((p2.row.Q, old.V), (p2.col.Q, old.W)):
            Qf, Kf = new.full(), kept.full()
            for c in range(tree.nclusters):
                K = Kf[c]
                if K.size == 0:
                    continue
                res = np.linalg.norm(K - Qf[c] @ (Qf[c].T @ K)) / np.linalg.norm(K)
                assert res <= 1e-12, (c, res)


def test_update_by_zero_product_keeps_target():
    """X = 0: Z + 0 X Y equals Z (to rounding) with the old ranks."""
    _, tree, bt, X, Y = problem("2d")
    _, p2a = O.multiply(X, Y, bt, 1e-6)
    _, p2 = O.multiply(O.scaled(X, 0.0), Y, bt, 1e-6, Zold=p2a.Z)
    assert relF(p2.Z.dense(), p2a.Z.dense()) <= 1e-13
    nc = tree.nclusters
    assert [p2.row.Q.rank[c] for c in range(nc)] == [p2a.row.Q.rank[c] for c in range(nc)]
    assert [p2.col.Q.rank[c] for c in range(nc)] == [p2a.col.Q.rank[c] for c in range(nc)]


# --------------------------------------------------------------------------
# R23 (variant of R9): level-dependent tolerances eps_l = eps zeta^(D - l)
# --------------------------------------------------------------------------
def test_level_eps_geometric_in_the_level():
    """Leaves get eps; each level towards the root multiplies it by zeta;
    zeta outside (0, 1] is refused."""
    _, tree, _, _, _ = problem("2d")
    eps, zeta = 1e-5, 0.3
    for c in range(tree.nclusters):
        e = OH.level_eps(eps, zeta, tree, c)
        if tree.is_leaf(c):
            assert e == eps
        for ch in tree.children[c]:
            assert np.isclose(OH.level_eps(eps, zeta, tree, ch) * zeta, e, rtol=1e-14)
    assert OH.level_eps(eps, zeta, tree, 0) == pytest.approx(eps * zeta ** tree.depth, rel=1e-14)
    for bad in (0.0, -0.5, 1.5):
        with pytest.raises(ValueError):
            OH.level_eps(eps, bad, tree, 0)


@pytest.mark.parametrize("name", ["1d", "2d"])
def test_level_factor_one_is_the_uniform_rule(name):
    _, tree, bt, X, Y = problem(name)
    p1, p2 = product(name, 1e-6)
    q1, q2 = O.multiply(X, Y, bt, 1e-6, zeta=1.0)
    nc = tree.nclusters
    for a, b in ((p1.row, q1.row), (p1.col, q1.col), (p2.row, q2.row), (p2.col, q2.col)):
        assert [a.Q.rank[c] for c in range(nc)] == [b.Q.rank[c] for c in range(nc)]
    assert np.array_equal(p2.Z.dense(), q2.Z.dense())


def _spectral(M):
    return np.linalg.norm(M, 2) if M.size else 0.0


@pytest.mark.parametrize("name,eps,zeta", [("1d", 1e-4, 0.5), ("2d", 1e-5, 0.25), ("2d", 1e-7, 0.5)])
def test_level_tolerance_truncation_of_each_cluster(name, eps, zeta):
    """Under R23 every truncation meets its own level's tolerance, checked
    from the matrices themselves: the projection residual of C_t (Chat_t)
    onto the new basis is at most eps_l in the spectral norm, and the rank is
    minimal (the smallest kept singular value of C_t exceeds eps_l); phase 1
    likewise for the remainder outside the kept range of V_X.  The leaf
    ranks of phase 1 equal those of the uniform rule (same eps, same input)."""
    _, tree, bt, X, Y = problem(name)
    p1, p2 = O.multiply(X, Y, bt, eps, zeta=zeta)
    u1, u2 = product(name, eps)
    D = tree.depth
    for side in (p2.row, p2.col):
        for t, C in side.C.items():
            if C.size == 0:
                continue
            el = eps * zeta ** (D - tree.level[t])
            Q = side.Q.leaf[t] if tree.is_leaf(t) else (
                _stacked_transfers(side.Q, tree, t) if side.Q.rank[t] else np.zeros((C.shape[0], 0)))
            assert _spectral(C - Q @ (Q.T @ C)) <= el * (1 + 1e-9) + 1e-13 * _spectral(C)
            sv = np.linalg.svd(C, compute_uv=False)
            k = Q.shape[1]
            assert k == 0 or sv[k - 1] > el * (1 - 1e-9)
    Qf = p1.row.Q.full()
    for t, (VX, Vrest) in p1.row.assembled.items():
        if Vrest.size == 0:
            continue
        el = eps * zeta ** (D - tree.level[t])
        Q = Qf[t] if tree.is_leaf(t) else _stacked_transfers(p1.row.Q, tree, t)
        Ux, sx, _ = np.linalg.svd(VX, full_matrices=True)
        k1 = int(np.count_nonzero(sx > OH.VX_RTOL * sx[0])) if sx.size and sx[0] > 0 else 0
        assert _spectral(Vrest - Q @ (Q.T @ Vrest)) <= el * (1 + 1e-9) + 1e-13 * _spectral(Vrest)
    for a, b in ((p1.row, u1.row), (p1.col, u1.col)):
        for t in tree.leaves:
            assert a.Q.rank[t] == b.Q.rank[t]
    # the tighter inner tolerances change some decision (the variant is active)
    nc = tree.nclusters
    assert any([a.Q.rank[c] for c in range(nc)] != [b.Q.rank[c] for c in range(nc)]
               for a, b in ((p1.row, u1.row), (p2.row, u2.row)))
