"""FP64 CPU oracle for adaptive H^2-matrix multiplication Z <- Z + X Y.

Source: S. Boerm, "Adaptive fast multiplication of H^2-matrices",
arXiv 2309.09061.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference the HIP path is checked against.  Only the tests, the smoke check of
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it.  It shares no code with the HIP path; both are fed by ``workloads.py``.

Everything is float64 numpy.  Library QR / SVD / matmul serve as single steps;
the loops over clusters and blocks follow the recursive procedures of the
paper (basis weights, total weights, induced basis, build basis, match
column) in the paper's order and notation.  Where the paper is silent the
reading used is named in the docstring (readings R1..R21).

Conventions: clusters are numbered breadth-first (root 0); all matrices are
indexed in cluster order (the permuted order of the points).  A cluster basis
stores leaf matrices and transfer matrices E_{t'} (rank(t') x rank(parent)).
"""
from __future__ import annotations

import numpy as np

ADM, INADM, SPLIT = "A", "I", "N"

# Relative tolerance of the numerical rank of V_{X,t} (reading R18).
VX_RTOL = 1e-12
# Section 5 scaling (reading R8): a block whose spectral norm is at most
# BLOCK_RTOL times the largest block norm of its level (same pass, same kind
# of block) is zero up to rounding and is dropped like a block of norm 0.
BLOCK_RTOL = 1e-12
# blocks dropped by that rule (not by an exact zero norm) since import
DROPPED = [0]


# ----------------------------------------------------------------------------
# Work ledger: algorithmic floating-point operations per step and kind,
# counted at every dense operation of the method (not of the checks):
#   gemm   2 m n k for each product of an m x k and a k x n matrix;
#   qr     Householder QR of an m x n matrix, 2 n^2 (m - n/3) for m >= n and
#          2 m^2 (n - m/3) otherwise; forming an explicit m x m orthogonal
#          factor from p reflectors adds 4 (m^2 p - m p^2 + p^3/3);
#   svd    an SVD is counted as the QR of the matrix (kind qr) followed by
#          the SVD of its p x p triangular factor, p = min(m, n): 12 p^3 for
#          the singular values with one set of singular vectors (Golub-Reinsch
#          counts, Golub and Van Loan, "Matrix Computations", 4th ed.,
#          Section 8.6);
#   norm   a spectral norm, the same with values only: 8 p^3 / 3 after the QR;
#   sumsq  2 per entry of a sum of squares.
# Steps: setup, p1_row, p1_col, p1_mat, p2_row, p2_col, p2_mat.
# ----------------------------------------------------------------------------
_LEDGER = None
_STAGE = ["other"]


class counting:
    """``with counting() as ledger:`` collects {(step, kind): flops} of the
    oracle calls made inside the block."""

    def __enter__(self):
        global _LEDGER
        self.prev = _LEDGER
        _LEDGER = {}
        self.ledger = _LEDGER
        return self.ledger

    def __exit__(self, *exc):
        global _LEDGER
        _LEDGER = self.prev
        return False


class _stage:
    def __init__(self, name):
        self.name = name

    def __enter__(self):
        _STAGE.append(self.name)

    def __exit__(self, *exc):
        _STAGE.pop()
        return False


def _count(kind: str, flops: float):
    if _LEDGER is not None:
        key = (_STAGE[-1], kind)
        _LEDGER[key] = _LEDGER.get(key, 0.0) + float(flops)


def _qr_flops(m: int, n: int) -> float:
    if m >= n:
        return 2.0 * n * n * (m - n / 3.0)
    return 2.0 * m * m * (n - m / 3.0)


def mul(*factors: np.ndarray) -> np.ndarray:
    """Product of the factors from left to right, counted in the ledger."""
    out = factors[0]
    for f in factors[1:]:
        _count("gemm", 2.0 * out.shape[0] * out.shape[1] * f.shape[1])
        out = out @ f
    return out


# ----------------------------------------------------------------------------
# Cluster tree (Section 2, Definition "Cluster tree"; readings R1, R2)
# ----------------------------------------------------------------------------
class ClusterTree:
    """Binary cluster tree of uniform depth built by median bisection.

    R1: a cluster is split along the longest edge of the tight bounding box of
    its points (lowest axis on ties) at the median of (coordinate, original
    index); the first floor(m/2) points form child 0.  Every branch is split
    down to the common depth D = min{D >= 0 : leaf_size * 2**D >= n}.
    R2: boxes are tight axis-aligned boxes of the cluster's points.
    """

    def __init__(self, points: np.ndarray, leaf_size: int):
        pts = np.asarray(points, dtype=np.float64)
        if pts.ndim == 1:
            pts = pts[:, None]
        n, d = pts.shape
        if leaf_size < 2:
            raise ValueError("leaf_size must be >= 2")
        depth = 0
        while leaf_size * (1 << depth) < n:
            depth += 1
        self.n, self.dim, self.depth = n, d, depth
        # level by level, breadth first
        idx_lists = [np.arange(n)]
        level_of = [0]
        parent = [-1]
        children: list[list[int]] = [[]]
        for lev in range(depth):
            first = (1 << lev) - 1
            for c in range(first, first + (1 << lev)):
                idx = idx_lists[c]
                sub = pts[idx]
                ext = sub.max(axis=0) - sub.min(axis=0)
                ax = int(np.argmax(ext))
                order = np.lexsort((idx, sub[:, ax]))   # primary: coordinate, secondary: index
                srt = idx[order]
                h = len(srt) // 2
                for part in (srt[:h], srt[h:]):
                    children[c].append(len(idx_lists))
                    idx_lists.append(part)
                    level_of.append(lev + 1)
                    parent.append(c)
                    children.append([])
        nc = len(idx_lists)
        self.nclusters = nc
        self.parent = parent
        self.children = children
        self.level = level_of
        leaves = [c for c in range(nc) if not children[c]]
        self.perm = np.concatenate([idx_lists[c] for c in leaves]) if leaves else np.zeros(0, int)
        # offsets in permuted order
        self.off = np.zeros(nc, dtype=np.int64)
        self.size = np.array([len(x) for x in idx_lists], dtype=np.int64)
        pos = 0
        for c in leaves:
            self.off[c] = pos
            pos += self.size[c]
        for c in range(nc - 1, -1, -1):
            if children[c]:
                self.off[c] = self.off[children[c][0]]
        self.points = pts[self.perm]             # permuted points
        self.bmin = np.array([pts[idx].min(axis=0) for idx in idx_lists])
        self.bmax = np.array([pts[idx].max(axis=0) for idx in idx_lists])
        self.leaves = leaves

    def is_leaf(self, c: int) -> bool:
        return not self.children[c]

    def rng(self, c: int) -> slice:
        return slice(int(self.off[c]), int(self.off[c] + self.size[c]))

    def diam(self, c: int) -> float:
        return float(np.linalg.norm(self.bmax[c] - self.bmin[c]))

    def dist(self, a: int, b: int) -> float:
        gap = np.maximum(0.0, np.maximum(self.bmin[b] - self.bmax[a], self.bmin[a] - self.bmax[b]))
        return float(np.linalg.norm(gap))

    def clusters_at(self, lev: int):
        return range((1 << lev) - 1, (1 << (lev + 1)) - 1)


# ----------------------------------------------------------------------------
# Block tree (Section 2, Definition "Block tree"; reading R3)
# ----------------------------------------------------------------------------
class BlockTree:
    """Block tree for (row tree, column tree) with standard admissibility.

    R3: (t,s) is admissible iff dist(B_t, B_s) > 0 and
    max(diam B_t, diam B_s) <= eta * dist(B_t, B_s).  Blocks are refined from
    (root, root) by the children rule of the definition and refinement stops
    at admissible blocks or leaf x leaf blocks.
    """

    def __init__(self, rt: ClusterTree, ct: ClusterTree, eta: float, types=None, children=None):
        self.rt, self.ct, self.eta = rt, ct, eta
        if types is not None:
            self.type, self.children = types, children
            return
        self.type: dict = {}
        self.children: dict = {}
        stack = [(0, 0)]
        while stack:
            t, s = stack.pop()
            if self.admissible(t, s):
                self.type[(t, s)] = ADM
                self.children[(t, s)] = []
                continue
            ct_, cs_ = rt.children[t], ct.children[s]
            if not ct_ and not cs_:
                self.type[(t, s)] = INADM
                self.children[(t, s)] = []
                continue
            self.type[(t, s)] = SPLIT
            tl = ct_ if ct_ else [t]
            sl = cs_ if cs_ else [s]
            kids = [(a, b) for a in tl for b in sl]
            self.children[(t, s)] = kids
            stack.extend(kids)

    def admissible(self, t: int, s: int) -> bool:
        dist = self.rt.dist_to(self.ct, t, s) if self.rt is not self.ct else self.rt.dist(t, s)
        if dist <= 0.0:
            return False
        return max(self.rt.diam(t), self.ct.diam(s)) <= self.eta * dist

    def leaves(self, typ=None):
        return [b for b, ty in self.type.items() if ty != SPLIT and (typ is None or ty == typ)]

    def transposed(self) -> "BlockTree":
        types = {(s, t): ty for (t, s), ty in self.type.items()}
        kids = {(s, t): [(b, a) for (a, b) in ch] for (t, s), ch in self.children.items()}
        return BlockTree(self.ct, self.rt, self.eta, types, kids)

    def row_map(self, typ):
        """t -> sorted list of s with (t,s) of the given type(s)."""
        out: dict = {}
        for (t, s), ty in self.type.items():
            if ty in typ:
                out.setdefault(t, []).append(s)
        for v in out.values():
            v.sort()
        return out


def _dist_to(self, other, a, b):
    gap = np.maximum(0.0, np.maximum(other.bmin[b] - self.bmax[a], self.bmin[a] - other.bmax[b]))
    return float(np.linalg.norm(gap))


ClusterTree.dist_to = _dist_to


# ----------------------------------------------------------------------------
# Cluster bases and H^2-matrices (Section 2, Definitions "Cluster basis",
# "H^2-matrix", eq. (vsw), eq. (transfer))
# ----------------------------------------------------------------------------
class ClusterBasis:
    """Nested cluster basis: leaf matrices and transfer matrices E_{t'}."""

    def __init__(self, tree: ClusterTree):
        self.tree = tree
        self.rank: dict = {}
        self.leaf: dict = {}       # leaf t -> (#t x rank(t))
        self.transfer: dict = {}   # non-root t -> (rank(t) x rank(parent))

    def full(self) -> dict:
        """Expanded V_t for every cluster (V_t|_{t'} = V_{t'} E_{t'})."""
        tr = self.tree
        out = {}
        for c in range(tr.nclusters - 1, -1, -1):
            if tr.is_leaf(c):
                out[c] = self.leaf[c]
            else:
                out[c] = np.vstack([out[ch] @ self.transfer[ch] for ch in tr.children[c]])
        return out


class H2Matrix:
    """H^2-matrix: row basis V, column basis W, couplings S on admissible
    leaves, dense nearfield N on inadmissible leaves (Definition "H^2-matrix")."""

    def __init__(self, V: ClusterBasis, W: ClusterBasis, bt: BlockTree, S: dict, N: dict):
        self.V, self.W, self.bt, self.S, self.N = V, W, bt, S, N

    @property
    def shape(self):
        return (self.V.tree.n, self.W.tree.n)

    def transposed(self) -> "H2Matrix":
        return H2Matrix(self.W, self.V, self.bt.transposed(),
                        {(s, t): m.T for (t, s), m in self.S.items()},
                        {(s, t): m.T for (t, s), m in self.N.items()})

    def dense(self) -> np.ndarray:
        rt, ct = self.V.tree, self.W.tree
        Vf, Wf = self.V.full(), self.W.full()
        out = np.zeros((rt.n, ct.n))
        for (t, s), m in self.S.items():
            out[rt.rng(t), ct.rng(s)] = Vf[t] @ m @ Wf[s].T
        for (t, s), m in self.N.items():
            out[rt.rng(t), ct.rng(s)] = m
        return out

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x in O(nk) (forward transform, couplings, backward transform,
        nearfield); x is n x p in cluster order."""
        rt, ct = self.V.tree, self.W.tree
        x = np.asarray(x, dtype=np.float64)
        vec = x.ndim == 1
        if vec:
            x = x[:, None]
        xh = {}
        for c in range(ct.nclusters - 1, -1, -1):
            if ct.is_leaf(c):
                xh[c] = self.W.leaf[c].T @ x[ct.rng(c)]
            else:
                xh[c] = sum(self.W.transfer[ch].T @ xh[ch] for ch in ct.children[c])
        yh = {c: np.zeros((self.V.rank[c], x.shape[1])) for c in range(rt.nclusters)}
        for (t, s), m in self.S.items():
            yh[t] += m @ xh[s]
        y = np.zeros((rt.n, x.shape[1]))
        for c in range(rt.nclusters):
            if c > 0:
                yh[c] += self.V.transfer[c] @ yh[rt.parent[c]]
            if rt.is_leaf(c):
                y[rt.rng(c)] += self.V.leaf[c] @ yh[c]
        for (t, s), m in self.N.items():
            y[rt.rng(t)] += m @ x[ct.rng(s)]
        return y[:, 0] if vec else y


# ----------------------------------------------------------------------------
# Construction by Chebyshev interpolation (Section 2, Example "Integral
# operator"; readings R4, R5)
# ----------------------------------------------------------------------------
def kernel_eval(kind: str, x: np.ndarray, y: np.ndarray, same_index=None, nx: np.ndarray = None) -> np.ndarray:
    """g(x_i, y_j) for point arrays x (p x d), y (q x d).  R5: entries with
    i == j (same_index given as the diagonal offset) use the diagonal rule.
    The double-layer kernel "dlp" of Section 7, <n(x), x - y> / (4 pi |x - y|^3),
    takes the unit normals nx (p x d) at the points x."""
    diff = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=2))
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == "dlp":
            g, dg = np.sum(nx[:, None, :] * diff, axis=2) / (4.0 * np.pi * r ** 3), 0.0
        elif kind == "log":
            g, dg = np.log(r), 0.0
        elif kind == "expneg":
            g, dg = np.exp(-r), 1.0
        elif kind == "inv4pi":
            g, dg = 1.0 / (4.0 * np.pi * r), 0.0
        elif kind == "inv":
            g, dg = 1.0 / r, 0.0
        elif kind == "poly2":
            g, dg = (x @ y.T) ** 2, None
        else:
            raise ValueError(kind)
    if same_index is not None and dg is not None:
        m = min(x.shape[0], y.shape[0])
        g[np.arange(m), np.arange(m)] = dg
    return g


def cheb_nodes(a: float, b: float, m: int) -> np.ndarray:
    """Chebyshev points cos((2j-1) pi / (2m)), j = 1..m, mapped to [a, b]."""
    j = np.arange(1, m + 1)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * j - 1) * np.pi / (2 * m))


def lagrange(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[i, j] = prod_{q != j} (x_i - xi_q) / (xi_j - xi_q)."""
    m = len(nodes)
    L = np.ones((len(x), m))
    for j in range(m):
        for q in range(m):
            if q != j:
                L[:, j] *= (x - nodes[q]) / (nodes[j] - nodes[q])
    return L


def lagrange_derivative(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[i, j] = l_j'(x_i), written without division by x - xi:
    l_j'(x) = sum_{q != j} 1/(xi_j - xi_q) prod_{r != j, q} (x - xi_r)/(xi_j - xi_r)."""
    m = len(nodes)
    D = np.zeros((len(x), m))
    for j in range(m):
        for q in range(m):
            if q == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[q]))
            for r_ in range(m):
                if r_ != j and r_ != q:
                    term *= (x - nodes[r_]) / (nodes[j] - nodes[r_])
            D[:, j] += term
    return D


def _axis_boxes(tree: ClusterTree, c: int):
    """R4: box edges narrower than 1e-12 * root diameter are widened."""
    floor = 1e-12 * tree.diam(0)
    lo, hi = tree.bmin[c].copy(), tree.bmax[c].copy()
    for a in range(tree.dim):
        w = hi[a] - lo[a]
        if w < floor:
            mid = 0.5 * (lo[a] + hi[a])
            lo[a], hi[a] = mid - 0.5 * floor, mid + 0.5 * floor
    return lo, hi


def _cube_boxes(tree: ClusterTree, c: int):
    """R22: interpolation box of the double-layer bases, the bounding cube of
    the cluster's (R4-widened) box: same center, every edge as long as the
    longest.  A cluster on one face of the cube surface has a flat box, on
    which derivatives across the face would be determined by rounding."""
    lo, hi = _axis_boxes(tree, c)
    half = 0.5 * float(np.max(hi - lo))
    mid = 0.5 * (lo + hi)
    return mid - half, mid + half


def _multi_indices(m: int, d: int) -> np.ndarray:
    """Tensor multi-indices, axis 0 fastest: nu = nu_0 + m nu_1 + m^2 nu_2."""
    k = m ** d
    lin = np.arange(k)
    return np.stack([(lin // (m ** a)) % m for a in range(d)], axis=1)


def interpolation_points(tree: ClusterTree, c: int, m: int, boxes=_axis_boxes) -> np.ndarray:
    lo, hi = boxes(tree, c)
    mi = _multi_indices(m, tree.dim)
    nodes = [cheb_nodes(lo[a], hi[a], m) for a in range(tree.dim)]
    return np.stack([nodes[a][mi[:, a]] for a in range(tree.dim)], axis=1)


def _tensor_lagrange(tree: ClusterTree, c: int, m: int, x: np.ndarray, boxes=_axis_boxes) -> np.ndarray:
    """Tensor Lagrange polynomials of cluster c evaluated at points x (p x d)."""
    lo, hi = boxes(tree, c)
    mi = _multi_indices(m, tree.dim)
    out = np.ones((x.shape[0], m ** tree.dim))
    for a in range(tree.dim):
        La = lagrange(cheb_nodes(lo[a], hi[a], m), x[:, a])
        out *= La[:, mi[:, a]]
    return out


def _tensor_normal_derivative(tree: ClusterTree, c: int, m: int, x: np.ndarray, nx: np.ndarray,
                              boxes=_axis_boxes) -> np.ndarray:
    """-<n(x_i), grad l_{c,nu}(x_i)> for points x (p x d) with normals nx."""
    lo, hi = boxes(tree, c)
    mi = _multi_indices(m, tree.dim)
    L, D = [], []
    for a in range(tree.dim):
        nodes = cheb_nodes(lo[a], hi[a], m)
        L.append(lagrange(nodes, x[:, a])[:, mi[:, a]])
        D.append(lagrange_derivative(nodes, x[:, a])[:, mi[:, a]])
    out = np.zeros((x.shape[0], m ** tree.dim))
    for d in range(tree.dim):
        term = D[d].copy()
        for a in range(tree.dim):
            if a != d:
                term *= L[a]
        out -= nx[:, d:d + 1] * term
    return out


def interpolation_basis(tree: ClusterTree, m: int, boxes=_axis_boxes) -> ClusterBasis:
    """Leaf V_t[i,nu] = l_{t,nu}(x_i); transfer E_{t'}[nu',nu] = l_{t,nu}(xi_{t',nu'})."""
    cb = ClusterBasis(tree)
    k = m ** tree.dim
    for c in range(tree.nclusters):
        cb.rank[c] = k
        if tree.is_leaf(c):
            cb.leaf[c] = _tensor_lagrange(tree, c, m, tree.points[tree.rng(c)], boxes)
        if c > 0:
            cb.transfer[c] = _tensor_lagrange(tree, tree.parent[c], m, interpolation_points(tree, c, m, boxes),
                                              boxes)
    return cb


def normal_derivative_basis(tree: ClusterTree, m: int, normals: np.ndarray) -> ClusterBasis:
    """Row basis of the double-layer kernel: with gamma(x, y) = 1/(4 pi |x - y|),
    <n(x), x - y>/(4 pi |x - y|^3) = -<n(x), grad_x gamma(x, y)>, so the
    interpolant of gamma gives leaf V_t[i,nu] = -<n(x_i), grad l_{t,nu}(x_i)>;
    transfers as for the interpolation basis (the gradient of a nested
    polynomial is nested), on the R22 boxes.  normals: cluster order."""
    cb = interpolation_basis(tree, m, _cube_boxes)
    for c in tree.leaves:
        r = tree.rng(c)
        cb.leaf[c] = _tensor_normal_derivative(tree, c, m, tree.points[r], normals[r], _cube_boxes)
    return cb


def kernel_h2(tree: ClusterTree, bt: BlockTree, kind: str, m: int, basis: ClusterBasis = None) -> H2Matrix:
    """S_ts[nu,mu] = g(xi_{t,nu}, xi_{s,mu}) on admissible leaves; g(x_i, x_j)
    on inadmissible leaves; W = V (same interpolation on both sides)."""
    V = basis if basis is not None else interpolation_basis(tree, m)
    ip = {c: interpolation_points(tree, c, m) for c in range(tree.nclusters)}
    S, N = {}, {}
    for (t, s), ty in bt.type.items():
        if ty == ADM:
            S[(t, s)] = kernel_eval(kind, ip[t], ip[s])
        elif ty == INADM:
            N[(t, s)] = kernel_eval(kind, tree.points[tree.rng(t)], tree.points[tree.rng(s)],
                                    same_index=True if t == s else None)
    return H2Matrix(V, V, bt, S, N)


def dlp_h2(tree: ClusterTree, bt: BlockTree, m: int, normals: np.ndarray) -> H2Matrix:
    """The double-layer kernel matrix of Section 7 (<n(x_i), x_i - x_j> /
    (4 pi |x_i - x_j|^3), diagonal 0; normals in the input point order):
    row basis normal_derivative_basis, column basis the interpolation basis,
    both on the R22 boxes; S_ts[nu,mu] = gamma(xi_{t,nu}, xi_{s,mu}); exact
    nearfield.  Not symmetric: row and column bases differ."""
    nrm = np.asarray(normals, dtype=np.float64)[tree.perm]
    V = normal_derivative_basis(tree, m, nrm)
    Wb = interpolation_basis(tree, m, _cube_boxes)
    ip = {c: interpolation_points(tree, c, m, _cube_boxes) for c in range(tree.nclusters)}
    S, N = {}, {}
    for (t, s), ty in bt.type.items():
        if ty == ADM:
            S[(t, s)] = kernel_eval("inv4pi", ip[t], ip[s])
        elif ty == INADM:
            rt, rs = tree.rng(t), tree.rng(s)
            N[(t, s)] = kernel_eval("dlp", tree.points[rt], tree.points[rs], same_index=True if t == s else None,
                                    nx=nrm[rt])
    return H2Matrix(V, Wb, bt, S, N)


def identity_h2(tree: ClusterTree, bt: BlockTree, m: int) -> H2Matrix:
    """The identity as an H^2-matrix: zero couplings, identity diagonal blocks."""
    V = interpolation_basis(tree, m)
    k = m ** tree.dim
    S = {b: np.zeros((k, k)) for b, ty in bt.type.items() if ty == ADM}
    N = {}
    for (t, s), ty in bt.type.items():
        if ty == INADM:
            N[(t, s)] = np.eye(tree.size[t]) if t == s else np.zeros((tree.size[t], tree.size[s]))
    return H2Matrix(V, V, bt, S, N)


def scaled(A: H2Matrix, alpha: float) -> H2Matrix:
    return H2Matrix(A.V, A.W, A.bt, {b: alpha * m for b, m in A.S.items()},
                    {b: alpha * m for b, m in A.N.items()})


# ----------------------------------------------------------------------------
# Small dense helpers (library primitives)
# ----------------------------------------------------------------------------
def qr_r(M: np.ndarray) -> np.ndarray:
    """R factor of a thin Householder QR, min(rows, cols) x cols."""
    if M.shape[0] == 0:
        return np.zeros((0, M.shape[1]))
    _count("qr", _qr_flops(*M.shape))
    return np.linalg.qr(M, mode="r")


def norm2(M: np.ndarray) -> float:
    if M.size == 0:
        return 0.0
    p = min(M.shape)
    _count("qr", _qr_flops(*M.shape))
    _count("norm", 8.0 * p ** 3 / 3.0)
    return float(np.linalg.norm(M, 2))


def left_svd(M: np.ndarray):
    """Left singular vectors and singular values (descending)."""
    if M.shape[0] == 0 or M.shape[1] == 0:
        return np.zeros((M.shape[0], 0)), np.zeros(0)
    _count("qr", _qr_flops(*M.shape))
    _count("svd", 12.0 * min(M.shape) ** 3)
    U, sig, _ = np.linalg.svd(M, full_matrices=False)
    return U, sig


RANK_ABS, RANK_REL_FROB = "abs", "relF"


def choose_rank(sig: np.ndarray, eps: float, rule: str = RANK_ABS) -> int:
    """Rank of a truncated SVD with singular values sig (descending).

    R9 (rule "abs", the paper's): keep the singular values strictly above eps
    on the scaled matrix.
    R21 (rule "relF", a variant): the smallest k whose discarded tail has
    Frobenius norm at most eps times the Frobenius norm of the whole matrix,
    i.e. keep sigma_i while sqrt(sum_{j >= i} sigma_j^2) > eps ||sigma||_2.
    """
    if rule == RANK_ABS:
        return int(np.count_nonzero(sig > eps))
    if rule != RANK_REL_FROB:
        raise ValueError(f"unknown rank rule {rule!r}")
    if sig.size == 0:
        return 0
    tail = np.sqrt(np.cumsum((sig * sig)[::-1])[::-1])  # tail[i] = ||sig[i:]||_2
    return int(np.count_nonzero(tail > eps * tail[0]))


def level_eps(eps: float, zeta: float, tree: "ClusterTree", t: int) -> float:
    """R23 (variant, level-dependent tolerances): the truncation of cluster t
    uses eps_l = eps * zeta**(D - l), l the level of t and D the depth of the
    tree, 0 < zeta <= 1.  Leaves keep eps and each level above tightens it by
    zeta, so the truncation errors met on the way from the leaves to a block
    of any level sum to at most eps / (1 - zeta) (zeta < 1).  zeta = 1 is the
    paper's uniform tolerance."""
    if not 0.0 < zeta <= 1.0:
        raise ValueError("zeta must lie in (0, 1]")
    return eps * zeta ** (tree.depth - tree.level[t])


# ----------------------------------------------------------------------------
# Phase 1 set-up: basis weights, cluster basis products, total weights
# (Section 4)
# ----------------------------------------------------------------------------
def basis_weights(W: ClusterBasis) -> dict:
    """Figure "basis_weights": R_r with W_r = Q_r R_r, bottom-up.

    R6: the stacked matrix of a non-leaf is [R_{r'} F_{r'}] (eq. (transfer)).
    """
    tr = W.tree
    R = {}

    def rec(r):
        if tr.is_leaf(r):
            R[r] = qr_r(W.leaf[r])
        else:
            for ch in tr.children[r]:
                rec(ch)
            R[r] = qr_r(np.vstack([mul(R[ch], W.transfer[ch]) for ch in tr.children[r]]))

    rec(0)
    return R


def cluster_basis_products(WX: ClusterBasis, VY: ClusterBasis) -> dict:
    """P_{XY,s} = W_{X,s}^* V_{Y,s}; non-leaf: sum_{s'} F_{s'}^* P_{s'} E_{s'}."""
    tr = WX.tree
    P = {}
    for s in range(tr.nclusters - 1, -1, -1):
        if tr.is_leaf(s):
            P[s] = mul(WX.leaf[s].T, VY.leaf[s])
        else:
            P[s] = sum(mul(WX.transfer[ch].T, P[ch], VY.transfer[ch]) for ch in tr.children[s])
    return P


def total_weights(Y: H2Matrix, RY: dict) -> dict:
    """Figure "total_weights": Z_s = R factor of
    [Z_{s+} E_{Y,s}^*; R_{Y,r} S_{Y,sr}^* (r in row(s))], top-down.

    Section 5 / R8: block r is scaled by 1/||S_{Y,sr} R_{Y,r}^*||_2; blocks of
    norm zero, or at most BLOCK_RTOL times the largest of the level, are
    dropped.  R7: parent block first, then row(s) in increasing cluster id.
    The recursion is taken level by level from the root (the clusters of a
    level are independent).
    """
    tr = Y.V.tree
    row = Y.bt.row_map((ADM,))
    Z = {}
    for lev in range(tr.depth + 1):
        cls = list(tr.clusters_at(lev))
        M = {(s, r): mul(RY[r], Y.S[(s, r)].T) for s in cls for r in row.get(s, [])}
        w = {b: norm2(m) for b, m in M.items()}
        floor = BLOCK_RTOL * max(w.values(), default=0.0)
        for s in cls:
            blocks = []
            if lev > 0:
                blocks.append(mul(Z[tr.parent[s]], Y.V.transfer[s].T))
            for r in row.get(s, []):
                if w[(s, r)] > floor:
                    blocks.append(M[(s, r)] / w[(s, r)])
                elif w[(s, r)] > 0.0:
                    DROPPED[0] += 1
            G = np.vstack(blocks) if blocks else np.zeros((0, Y.V.rank[s]))
            Z[s] = qr_r(G)
    return Z


# ----------------------------------------------------------------------------
# Phase 1: compressed induced row basis (Section 4, Figure "induced_basis";
# error control Section 5)
# ----------------------------------------------------------------------------
class InducedBasis:
    """Result of one pass of Figure "induced_basis": isometric nested basis
    Q, basis change R_X (Q_t^* V_{X,t} = [R_{X,t}; 0]) and auxiliaries
    A_{t,s} = Q_t^* X|_{t x s} V_{Y,s} for s in C_t."""

    def __init__(self, Q, RX, A, sigmas, assembled):
        self.Q, self.RX, self.A, self.sigmas = Q, RX, A, sigmas
        self.assembled = assembled      # t -> (VX or VXhat, scaled remainder blocks)


def _pad_rows(M: np.ndarray, rows: int) -> np.ndarray:
    out = np.zeros((rows, M.shape[1]))
    out[:M.shape[0]] = M
    return out


def induced_basis(X: H2Matrix, Y: H2Matrix, eps: float, rule: str = RANK_ABS, zeta: float = 1.0) -> InducedBasis:
    """Compressed induced row basis of the product X Y.

    R18: Q_{X,t} is a full orthogonal factor whose first k1 columns span the
    range of V_{X,t}; k1 is the numerical rank of V_{X,t} (singular values
    above VX_RTOL times the largest), which equals the paper's min(k, rows)
    whenever V_{X,t} has full numerical rank, and Q_{X,t} is taken from the
    SVD of V_{X,t} so that the kept range is unique; the remainder has
    (rows - k1) rows.  R8: the block of s is scaled by
    1/||X|_{t x s} V_{Y,s}||_2 (leaf) or 1/||Ahat_{t,s}||_2 (non-leaf);
    blocks of norm zero, or at most BLOCK_RTOL times the largest block norm
    of the level, are dropped (zero up to rounding: for the double-layer
    kernel the blocks of two clusters on one face of the cube).
    R9: rank k2 = #{sigma > eps} (R23: eps of the cluster's level).  The
    recursion of Figure "induced_basis"
    is taken level by level from the leaves (the clusters of a level are
    independent), so that each level's largest block norm is known.
    """
    rt = X.V.tree
    if any(rt.level[c] != rt.depth for c in rt.leaves):
        raise ValueError("oracle expects uniform-depth cluster trees (R1)")
    k = X.V.rank[0]
    with _stage("setup"):
        RY = basis_weights(Y.W)
        P = cluster_basis_products(X.W, Y.V)
        Z = total_weights(Y, RY)
    Cmap = X.bt.row_map((INADM, SPLIT))
    Q = ClusterBasis(rt)
    RX, A, sig_out, assembled = {}, {}, {}, {}

    def compress(t, VX, Vrest_blocks):
        """Keep the (numerical) range of V_X exactly, SVD of the remainder."""
        rows = VX.shape[0]
        pv = min(VX.shape)
        _count("qr", _qr_flops(*VX.shape) + 4.0 * (rows * rows * pv - rows * pv * pv + pv ** 3 / 3.0))
        _count("svd", 12.0 * pv ** 3)
        Ux, sx, _ = np.linalg.svd(VX, full_matrices=True)          # Ux: rows x rows
        k1 = int(np.count_nonzero(sx > VX_RTOL * sx[0])) if sx.size and sx[0] > 0 else 0
        RX[t] = mul(Ux[:, :k1].T, VX)                              # Q_{X,t}^* V_{X,t} = [R_{X,t}; 0]
        Vrest = np.hstack(Vrest_blocks) if Vrest_blocks else np.zeros((rows, 0))
        assembled[t] = (VX, Vrest)
        Vtil = mul(Ux[:, k1:].T, Vrest)
        U, sig = left_svd(Vtil)
        k2 = choose_rank(sig, level_eps(eps, zeta, rt, t), rule)
        sig_out[t] = sig
        Qt = np.hstack([Ux[:, :k1], mul(Ux[:, k1:], U[:, :k2])])
        Q.rank[t] = k1 + k2
        return Qt

    def level_blocks(t):
        """The blocks of t (leaf: X|_{t x s} V_{Y,s}; else Ahat_{t,s}), and
        for a non-leaf the stacked V_X part and the children's row offsets."""
        if rt.is_leaf(t):
            B = {}
            for s in Cmap.get(t, []):
                assert X.bt.type[(t, s)] == INADM
                B[s] = mul(X.N[(t, s)], Y.V.leaf[s])      # X|_{t x s} V_{Y,s}
            return B, X.V.leaf[t], None
        kids = rt.children[t]
        offs, o = {}, 0
        for ch in kids:
            offs[ch] = o
            o += Q.rank[ch]
        rows = o
        VXhat = np.zeros((rows, k))
        for ch in kids:
            VXhat[offs[ch]:offs[ch] + RX[ch].shape[0]] = mul(RX[ch], X.V.transfer[ch])
        Ahat = {}
        for s in Cmap.get(t, []):
            M = np.zeros((rows, k))
            for ch in kids:
                for sc in Y.V.tree.children[s]:
                    ty = X.bt.type[(ch, sc)]
                    if ty == ADM:        # A_{t',s'} = [R_{X,t'} S_{X,t's'} P_{XY,s'}; 0]
                        At = _pad_rows(mul(RX[ch], X.S[(ch, sc)], P[sc]), Q.rank[ch])
                    else:
                        At = A[(ch, sc)]
                    M[offs[ch]:offs[ch] + Q.rank[ch]] += mul(At, Y.V.transfer[sc])
            Ahat[s] = M
        return Ahat, VXhat, offs

    for lev in range(rt.depth, -1, -1):
        cls = list(rt.clusters_at(lev))
        parts = {t: level_blocks(t) for t in cls}
        w = {(t, s): norm2(M) for t in cls for s, M in parts[t][0].items()}
        floor = BLOCK_RTOL * max(w.values(), default=0.0)
        for t in cls:
            Bs, VX, offs = parts[t]
            blocks = []
            for s, M in Bs.items():
                if w[(t, s)] > floor and Z[s].shape[0] > 0:
                    blocks.append(mul(M, Z[s].T) / w[(t, s)])
                elif 0.0 < w[(t, s)] <= floor:
                    DROPPED[0] += 1
            Qt = compress(t, VX, blocks)
            if offs is None:
                Q.leaf[t] = Qt
            else:
                for ch in rt.children[t]:
                    Q.transfer[ch] = Qt[offs[ch]:offs[ch] + Q.rank[ch], :]
            for s, M in Bs.items():
                A[(t, s)] = mul(Qt.T, M)

    out = InducedBasis(Q, RX, A, sig_out, assembled)
    out.P = P
    return out


# ----------------------------------------------------------------------------
# Product block tree and the intermediate product G (Section 6 opening;
# readings R13, R14)
# ----------------------------------------------------------------------------
class ProductTree:
    """T^XY with the triples (t,s,r) reaching each block.

    kind of a terminated triple: "AA", "AN" ((t,s) admissible), "NA"
    ((s,r) admissible), "NN" (both inadmissible leaves); recursing triples
    (both factors subdivided) are listed in ``split``.
    """

    def __init__(self, X: H2Matrix, Y: H2Matrix):
        rt, mt, ct = X.V.tree, X.W.tree, Y.W.tree
        self.rt, self.ct = rt, ct
        self.type, self.children, self.triples, self.split = {}, {}, {}, {}
        todo = [((0, 0), [0])]
        while todo:
            (t, r), mids = todo.pop()
            term, rec = [], []
            for s in mids:
                tx, ty = X.bt.type[(t, s)], Y.bt.type[(s, r)]
                if tx == SPLIT and ty == SPLIT:
                    rec.append(s)
                elif tx == ADM and ty == ADM:
                    term.append((s, "AA"))
                elif tx == ADM:
                    term.append((s, "AN"))
                elif ty == ADM:
                    term.append((s, "NA"))
                else:
                    assert tx == INADM and ty == INADM
                    term.append((s, "NN"))
            self.triples[(t, r)] = term
            self.split[(t, r)] = rec
            if rec:
                self.type[(t, r)] = SPLIT
                kids = []
                for tc in rt.children[t]:
                    for rc in ct.children[r]:
                        sub = [sc for s in rec for sc in mt.children[s]
                               if (tc, sc) in X.bt.type and (sc, rc) in Y.bt.type]
                        kids.append((tc, rc))
                        todo.append(((tc, rc), sub))
                self.children[(t, r)] = kids
            else:
                nn = any(kd == "NN" for _, kd in term)
                self.type[(t, r)] = INADM if nn else ADM
                self.children[(t, r)] = []
        self.bt = BlockTree(rt, ct, None, self.type, self.children)


def form_product(X: H2Matrix, Y: H2Matrix, rowb: InducedBasis, colb: InducedBasis, PT: ProductTree):
    """R14: G = sum over terminated triples of P_row X|_{ts} Y|_{sr} P_col,
    P_row = Q_t Q_t^* unless (t,s) is admissible, P_col = Q^W_r Q^W_r^* unless
    (s,r) is admissible, written in coefficients of (Q, Q^W) at the triple's
    block and pushed to the leaves of T^XY through the transfer matrices."""
    Q, QW = rowb.Q, colb.Q
    k = X.V.rank[0]
    P = rowb.P                          # P_{XY,s} of the row pass's set-up
    RXp = {t: _pad_rows(rowb.RX[t], Q.rank[t]) for t in rowb.RX}          # [R_{X,t}; 0]
    Rcp = {r: _pad_rows(colb.RX[r], QW.rank[r]) for r in colb.RX}         # [R^c_{Y,r}; 0]
    acc, S, N = {}, {}, {}
    order = [(0, 0)]
    parent = {}
    for b in order:          # breadth-first: parents before children
        for ch in PT.children[b]:
            parent[ch] = b
            order.append(ch)
    for (t, r) in order:
        M = np.zeros((Q.rank[t], QW.rank[r]))
        if (t, r) in parent:
            tp, rp = parent[(t, r)]
            M += mul(Q.transfer[t], acc[(tp, rp)], QW.transfer[r].T)
        dense = None
        for s, kd in PT.triples[(t, r)]:
            if kd == "NA":
                M += mul(rowb.A[(t, s)], Y.S[(s, r)], Rcp[r].T)
            elif kd == "AN":
                M += mul(RXp[t], X.S[(t, s)], colb.A[(r, s)].T)
            elif kd == "AA":
                M += mul(RXp[t], X.S[(t, s)], P[s], Y.S[(s, r)], Rcp[r].T)
            else:
                d = mul(X.N[(t, s)], Y.N[(s, r)])
                dense = d if dense is None else dense + d
        acc[(t, r)] = M
        ty = PT.type[(t, r)]
        if ty == ADM:
            S[(t, r)] = M
        elif ty == INADM:
            Nm = mul(Q.leaf[t], M, QW.leaf[r].T)
            N[(t, r)] = Nm + dense if dense is not None else Nm
    return H2Matrix(Q, QW, PT.bt, S, N)


class Phase1:
    def __init__(self, X, Y, eps, rule=RANK_ABS, zeta=1.0):
        with _stage("p1_row"):
            self.row = induced_basis(X, Y, eps, rule, zeta)
        with _stage("p1_col"):
            self.col = induced_basis(Y.transposed(), X.transposed(), eps, rule, zeta)
        with _stage("p1_mat"):
            self.PT = ProductTree(X, Y)
            self.G = form_product(X, Y, self.row, self.col, self.PT)


# ----------------------------------------------------------------------------
# Phase 2: coarsening into the prescribed block tree T_IK (Section 6;
# Figures "match_column" and "basis"; readings R10, R11, R12, R15, R19)
# ----------------------------------------------------------------------------
def tag_blocks(G: H2Matrix, TIK: BlockTree):
    """For every block of T^XY the leaf of T_IK containing it (None if the
    block is a non-leaf of T_IK).  Raises if T^XY does not refine T_IK."""
    tag = {}
    rt, ct = G.V.tree, G.W.tree

    def anc_or_self(t, lev):
        while rt.level[t] > lev:
            t = rt.parent[t]
        return t

    def anc_or_self_c(r, lev):
        while ct.level[r] > lev:
            r = ct.parent[r]
        return r

    for (t, r), ty in G.bt.type.items():
        found = None
        for lev in range(rt.level[t], -1, -1):
            b = (anc_or_self(t, lev), anc_or_self_c(r, lev))
            if b in TIK.type and TIK.type[b] != SPLIT:
                found = b
                break
        tag[(t, r)] = found
        if ty != SPLIT and found is None:
            raise ValueError("T^XY does not refine T_IK")
    return tag


def block_norms(G: H2Matrix, TIK: BlockTree, tag) -> dict:
    """R10: omega_b = 1/||G|_b||_F for admissible b of T_IK (isometric bases:
    sum of ||S||_F^2 and ||N||_F^2 of the T^XY leaves inside b)."""
    sq = {}
    for b, m in list(G.S.items()) + list(G.N.items()):
        tb = tag[b]
        if tb is not None and TIK.type[tb] == ADM:
            _count("sumsq", 2.0 * m.size)
            sq[tb] = sq.get(tb, 0.0) + float(np.sum(m * m))
    return {b: (1.0 / np.sqrt(v) if v > 0 else 0.0) for b, v in sq.items()}


class ColumnTree:
    """Column tree T_{(t,r)} (Definition "Column tree"): node -> children,
    leaf -> admissible flag."""

    def __init__(self, root):
        self.root = root
        self.kids = {root: []}
        self.adm = {}

    def leaves(self, ct: ClusterTree):
        out = []

        def walk(r):
            if self.kids[r]:
                for c in self.kids[r]:
                    walk(c)
            else:
                out.append(r)

        walk(self.root)
        return out


def column_trees(G: H2Matrix):
    """Column trees of all blocks of T^XY, bottom-up: the projection of the
    subtree rooted at (t,r) onto its column cluster."""
    ct = G.W.tree
    out = {}
    blocks = sorted(G.bt.type, key=lambda b: -G.V.tree.level[b[0]])
    for b in blocks:
        r = b[1]
        T = ColumnTree(r)
        ty = G.bt.type[b]
        if ty != SPLIT:
            T.adm[r] = ty == ADM
        else:
            T.kids[r] = list(ct.children[r])
            for ch in G.bt.children[b]:
                _union(T, out[ch])
        out[b] = T
    return out


def _union(T: ColumnTree, sub: ColumnTree):
    """Union of column trees: a node is a leaf only if it is a leaf in every
    tree containing it; a leaf is inadmissible if it is inadmissible in any."""
    for node, kids in sub.kids.items():
        if node not in T.kids:
            T.kids[node] = list(kids)
            if not kids:
                T.adm[node] = sub.adm[node]
        elif kids and not T.kids[node]:
            T.kids[node] = list(kids)
            T.adm.pop(node, None)
        elif not kids and not T.kids[node]:
            T.adm[node] = T.adm[node] and sub.adm[node]


def match_column(rep: dict, target: ColumnTree, W: ClusterBasis) -> dict:
    """Figure "match_column": bring a representation {leaf r: (adm, A_r)} of
    G|_{t x r} (G|_{t x r*} = A_{r*} W_{r*}^* on admissible leaves, explicit
    columns on inadmissible ones) onto the column tree ``target``:
    A_{r'} = A_r F_{r'}^* where the target refines an admissible leaf,
    A_r <- A_r W_r^* where an admissible leaf becomes inadmissible.
    R19: an inadmissible leaf is never refined (uniform-depth trees)."""
    out = {}

    def visit(r, adm, M):
        if target.kids.get(r):
            if not adm:
                raise ValueError("inadmissible column leaf refined by the target")
            for rc in target.kids[r]:
                visit(rc, True, mul(M, W.transfer[rc].T))
        else:
            tadm = target.adm[r]
            if adm and not tadm:
                M = mul(M, W.leaf[r].T)
            out[r] = (tadm, M)

    for r, (adm, M) in rep.items():
        visit(r, adm, M)
    return out


class CoarseBasis:
    def __init__(self, Q, R, A, sigmas, omega, tag, Z, C, RZ=None):
        self.Q, self.R, self.A, self.sigmas, self.omega, self.tag = Q, R, A, sigmas, omega, tag
        self.Z, self.C = Z, C           # product total weights, condensed C_t / Chat_t
        self.RZ = RZ                    # Z <- Z + X Y: Q_t^* V^Z_t, the old basis in the new one


def build_basis(G: H2Matrix, TIK: BlockTree, eps: float, rule: str = RANK_ABS,
                Vold: ClusterBasis = None, zeta: float = 1.0) -> CoarseBasis:
    """Figure "basis": adaptive isometric nested row basis for the coarse
    block tree T_IK, with the product total weights Z_t of
    eq. (Zt_condensation), leaf matrices C_t (eq. (ct_leaf)) and non-leaf
    matrices Chat_t (eq. (ct_nonleaf)).

    R11: only admissible leaves of T^XY inside admissible leaves of T_IK
    enter Z_t.  R12: "admissible ancestor in T_IK" includes the block itself.
    R10: every block lying in b of T_IK is scaled by omega_b.  R9: rank
    #{sigma > eps}.  R_t = Q_t^* V_t is the basis change from G's row basis.

    Z <- Z + X Y with Z != 0 (reading R16): Vold is the row basis of the
    old Z on T_IK.  Its range is kept exactly, as phase 1 keeps range(V_X)
    (Section 4, leaf case): at every cluster the new basis is an orthonormal
    basis of that range (numerical rank, VX_RTOL) followed by the truncated
    SVD of the part of C_t (or Chat_t) outside it; at a non-leaf the old
    basis enters through Vhat^Z_t = [RZ_{t'} E^Z_{t'}] with RZ_{t'} =
    Q_{t'}^* V^Z_{t'}.  The old Z is then represented exactly and only G is
    compressed, with G's block weights.
    """
    rt, ct = G.V.tree, G.W.tree
    tag = tag_blocks(G, TIK)
    omega = block_norms(G, TIK, tag)
    ctrees = column_trees(G)

    def in_adm(b):
        tb = tag[b]
        return tb is not None and TIK.type[tb] == ADM

    rowXY: dict = {}
    for b, ty in G.bt.type.items():
        rowXY.setdefault(b[0], []).append(b[1])
    for v in rowXY.values():
        v.sort()
    Q = ClusterBasis(rt)
    R, A, sig_out, Z, Cm, RZ = {}, {}, {}, {}, {}, {}

    def truncate(t, C, VZ):
        """Orthonormal basis of C_t truncated at eps; with VZ the exact range
        of VZ followed by the truncated part of C_t outside it."""
        eps_t = level_eps(eps, zeta, rt, t)
        if VZ is None:
            U, sig = left_svd(C)
            kz = choose_rank(sig, eps_t, rule)
            sig_out[t] = sig
            return U[:, :kz]
        rows = VZ.shape[0]
        pv = min(VZ.shape)
        _count("qr", _qr_flops(*VZ.shape) + 4.0 * (rows * rows * pv - rows * pv * pv + pv ** 3 / 3.0))
        _count("svd", 12.0 * pv ** 3)
        if VZ.shape[1] == 0:
            Ux, sx = np.eye(rows), np.zeros(0)
        else:
            Ux, sx, _ = np.linalg.svd(VZ, full_matrices=True)
        k1 = int(np.count_nonzero(sx > VX_RTOL * sx[0])) if sx.size and sx[0] > 0 else 0
        U, sig = left_svd(mul(Ux[:, k1:].T, C))
        k2 = choose_rank(sig, eps_t, rule)
        sig_out[t] = sig
        return np.hstack([Ux[:, :k1], mul(Ux[:, k1:], U[:, :k2])])

    def rep_of_child(tc, rc):
        ty = G.bt.type[(tc, rc)]
        if ty == ADM:
            return {rc: (True, mul(R[tc], G.S[(tc, rc)]))}
        return A[(tc, rc)]

    def rec(t, Zp):
        # total weights of the product (top-down part of the recursion)
        blocks = []
        if Zp is not None:
            blocks.append(mul(Zp, G.V.transfer[t].T))
        for r in rowXY.get(t, []):
            if G.bt.type[(t, r)] == ADM and in_adm((t, r)):
                blocks.append(omega[tag[(t, r)]] * G.S[(t, r)].T)
        Zt = qr_r(np.vstack(blocks)) if blocks else np.zeros((0, G.V.rank[t]))
        Z[t] = Zt
        if rt.is_leaf(t):
            cols = [mul(G.V.leaf[t], Zt.T)]
            inad = [r for r in rowXY.get(t, []) if G.bt.type[(t, r)] == INADM and in_adm((t, r))]
            for r in inad:
                cols.append(omega[tag[(t, r)]] * G.N[(t, r)])
            Cm[t] = np.hstack(cols)
            Qt = truncate(t, Cm[t], Vold.leaf[t] if Vold is not None else None)
            kz = Qt.shape[1]
            Q.leaf[t] = Qt
            Q.rank[t] = kz
            R[t] = mul(Qt.T, G.V.leaf[t])
            if Vold is not None:
                RZ[t] = mul(Qt.T, Vold.leaf[t])
            for r in inad:
                A[(t, r)] = {r: (False, mul(Qt.T, G.N[(t, r)]))}
            return
        kids = rt.children[t]
        for ch in kids:
            rec(ch, Zt)
        offs, o = {}, 0
        for ch in kids:
            offs[ch] = o
            o += Q.rank[ch]
        rows = o
        Vhat = np.zeros((rows, G.V.rank[t]))
        for ch in kids:
            Vhat[offs[ch]:offs[ch] + Q.rank[ch]] = mul(R[ch], G.V.transfer[ch])
        cols = [mul(Vhat, Zt.T)]
        split = [r for r in rowXY.get(t, []) if G.bt.type[(t, r)] == SPLIT and in_adm((t, r))]
        Ahat = {}
        for r in split:
            T = ctrees[(t, r)]
            leaves = T.leaves(ct)
            pieces = {}
            for tc in kids:
                merged = {}
                for rc in ct.children[r]:
                    merged.update(match_column(rep_of_child(tc, rc), T, G.W))
                for lf in leaves:
                    adm, M = merged[lf]
                    pieces.setdefault(lf, []).append(M)
            Ahat[r] = [(lf, T.adm[lf], np.vstack(pieces[lf])) for lf in leaves]
            cols.append(omega[tag[(t, r)]] * np.hstack([M for _, _, M in Ahat[r]]))
        Cm[t] = np.hstack(cols)
        VZhat = None
        if Vold is not None:
            VZhat = np.zeros((rows, Vold.rank[t]))
            for ch in kids:
                VZhat[offs[ch]:offs[ch] + Q.rank[ch]] = mul(RZ[ch], Vold.transfer[ch])
        Qhat = truncate(t, Cm[t], VZhat)
        kz = Qhat.shape[1]
        Q.rank[t] = kz
        if Vold is not None:
            RZ[t] = mul(Qhat.T, VZhat)
        for ch in kids:
            Q.transfer[ch] = Qhat[offs[ch]:offs[ch] + Q.rank[ch], :]
        R[t] = mul(Qhat.T, Vhat)
        for r in split:
            A[(t, r)] = {lf: (adm, mul(Qhat.T, M)) for lf, adm, M in Ahat[r]}

    rec(0, None)
    return CoarseBasis(Q, R, A, sig_out, omega, tag, Z, Cm, RZ if Vold is not None else None)


def form_coarse(G: H2Matrix, TIK: BlockTree, rowc: CoarseBasis, colc: CoarseBasis, Zold: H2Matrix = None) -> H2Matrix:
    """R15: Z = sum_{b in L+_IK} Q^Z Q^Z* G|_b Q^ZW Q^ZW* + sum_{b in L-_IK} G|_b,
    plus the old Z when it is not zero (R16: its couplings written in the new
    bases, RZ S^Z_b RZW^*, exact because its ranges are kept; its nearfield
    added).

    Couplings Q^Z_t^* G|_b Q^ZW_r are accumulated bottom-up over the blocks of
    T^XY inside b: R_t S_tr R^W_r^* on admissible leaves, Q^Z_t^* N_tr Q^ZW_r
    on inadmissible leaves, E^Z_{t'}^* L_{t'r'} F^Z_{r'} from children."""
    QZ, QZW = rowc.Q, colc.Q
    tag = rowc.tag
    L = {}
    blocks = sorted(G.bt.type, key=lambda b: -G.V.tree.level[b[0]])
    for b in blocks:
        tb = tag[b]
        if tb is None or TIK.type[tb] != ADM:
            continue
        t, r = b
        ty = G.bt.type[b]
        if ty == ADM:
            L[b] = mul(rowc.R[t], G.S[b], colc.R[r].T)
        elif ty == INADM:
            L[b] = mul(QZ.leaf[t].T, G.N[b], QZW.leaf[r])
        else:
            L[b] = sum(mul(QZ.transfer[tc].T, L[(tc, rc)], QZW.transfer[rc])
                       for (tc, rc) in G.bt.children[b])
    S, N = {}, {}
    for b, ty in TIK.type.items():
        if ty == ADM:
            S[b] = L[b] if b in L else np.zeros((QZ.rank[b[0]], QZW.rank[b[1]]))
            if Zold is not None:
                S[b] = S[b] + mul(rowc.RZ[b[0]], Zold.S[b], colc.RZ[b[1]].T)
        elif ty == INADM:
            gt = G.bt.type.get(b)
            if gt == INADM:
                N[b] = G.N[b]
            elif gt == ADM:
                N[b] = mul(G.V.leaf[b[0]], G.S[b], G.W.leaf[b[1]].T)
            else:
                raise ValueError("inadmissible leaf of T_IK not a leaf of T^XY")
            if Zold is not None:
                N[b] = N[b] + Zold.N[b]
    return H2Matrix(QZ, QZW, TIK, S, N)


class Phase2:
    """Z <- Z + G in T_IK; Zold (on T_IK) is the Z before the update, None
    for Z = 0."""

    def __init__(self, G: H2Matrix, TIK: BlockTree, eps: float, rule: str = RANK_ABS, Zold: H2Matrix = None,
                 zeta: float = 1.0):
        with _stage("p2_row"):
            self.row = build_basis(G, TIK, eps, rule, Zold.V if Zold is not None else None, zeta)
        with _stage("p2_col"):
            self.col = build_basis(G.transposed(), TIK.transposed(), eps, rule,
                                   Zold.W if Zold is not None else None, zeta)
        with _stage("p2_mat"):
            self.Z = form_coarse(G, TIK, self.row, self.col, Zold)


def multiply(X: H2Matrix, Y: H2Matrix, TIK: BlockTree, eps1: float, eps2: float = None, rule: str = RANK_ABS,
             Zold: H2Matrix = None, zeta: float = 1.0):
    """Both phases: returns (Phase1, Phase2); Z = phase2.Z approximates
    Zold + X Y (Zold on TIK, None for zero).  rule: the truncation rule of
    both phases (R9 "abs", or the variant R21 "relF"); zeta: the level
    factor of R23 (1: one tolerance on every level)."""
    p1 = Phase1(X, Y, eps1, rule, zeta)
    p2 = Phase2(p1.G, TIK, eps1 if eps2 is None else eps2, rule, Zold, zeta)
    return p1, p2


def build_problem(points, leaf_size, eta, order, kx, ky, normals=None):
    """Tree, block tree (T_IJ = T_JK = T_IK) and the H^2-matrices X, Y
    (kernel "dlp" needs the normals at the points, input order)."""
    tree = ClusterTree(points, leaf_size)
    bt = BlockTree(tree, tree, eta)
    V = interpolation_basis(tree, order) if "dlp" not in (kx, ky) or kx != ky else None

    def make(kind):
        return dlp_h2(tree, bt, order, normals) if kind == "dlp" else kernel_h2(tree, bt, kind, order, V)
    X = make(kx)
    Y = X if ky == kx else make(ky)
    return tree, bt, X, Y
