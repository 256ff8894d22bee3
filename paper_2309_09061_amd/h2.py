"""Python binding of the C-ABI in include/h2.h (argument marshalling only).

Every numerical step runs inside libh2.so (HIP kernels for gfx950).  Device
memory and streams come from PyTorch: vectors and dense outputs are
``torch.float64`` CUDA tensors, the context runs on
``torch.cuda.current_stream()``.  If libh2.so is missing the import fails;
there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2.so")

KERNELS = {"log": 0, "expneg": 1, "inv4pi": 2, "inv": 3, "dlp": 4, "poly2": 100}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16": 3}
KERNEL_FAMILIES = ["gemm_sum", "tsqr", "jacobi", "build", "other"]
STEPS = ["setup", "nearfield", "p1_row", "p1_col", "p1_mat", "p2_row", "p2_col", "p2_mat"]

_c_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def torch_allocator(device: int, stream: int):
    """Allocator callbacks backed by PyTorch's caching allocator on `device`
    and `stream` (what a Context uses by default)."""
    import torch

    def _alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:
            return None  # NULL: the library reports H2_ERR_ALLOC

    def _free(ptr, _user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass
    return ALLOC_FN(_alloc), FREE_FN(_free)


MAX_LEVELS = 32
HANDLE_KINDS = {"tree": 0, "matrix": 1, "product": 2}


class Stats(ctypes.Structure):
    """h2_stats_t of include/h2.h."""
    _fields_ = [(f, ctypes.c_int64) for f in ("n", "dim", "depth", "nclusters", "nblocks", "nadm", "ninadm",
                                               "triples", "device_bytes", "coupling_entries",
                                               "nearfield_entries")] + [
        ("rank_max", ctypes.c_int32 * 2), ("rank_mean", ctypes.c_double * 2),
        ("level_rank_max", (ctypes.c_int32 * MAX_LEVELS) * 2),
        ("level_rank_mean", (ctypes.c_double * MAX_LEVELS) * 2)]

    def as_dict(self) -> dict:
        out = {f: getattr(self, f) for f, _ in self._fields_[:11]}
        depth = int(self.depth)
        out["rank_max"] = list(self.rank_max)
        out["rank_mean"] = list(self.rank_mean)
        out["level_rank_max"] = [list(self.level_rank_max[w])[:depth + 1] for w in range(2)]
        out["level_rank_mean"] = [list(self.level_rank_mean[w])[:depth + 1] for w in range(2)]
        return out


def stats(obj) -> dict:
    """h2_stats of a Tree, Matrix or Product."""
    kind = {"Tree": 0, "Matrix": 1, "Product": 2}[type(obj).__name__]
    st = Stats()
    lib = obj.lib
    _check(lib, lib.h2_stats(obj.h, kind, ctypes.byref(st)))
    return st.as_dict()


def export(ctx, obj, path: str):
    """h2_export of a Tree, Matrix or Product into an .npz archive at path."""
    kind = {"Tree": 0, "Matrix": 1, "Product": 2}[type(obj).__name__]
    lib = obj.lib
    _check(lib, lib.h2_export(ctx.h if ctx is not None else None, obj.h, kind, os.fsencode(path)))


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"h2 status {code}: {msg}")
        self.code = code


def _declare(lib):
    sig = {
        "h2_last_error": (ctypes.c_char_p, []),
        "h2_ctx_create": (ctypes.c_int, [ctypes.c_int, _c_p, ALLOC_FN, FREE_FN, _c_p, ctypes.POINTER(_c_p)]),
        "h2_ctx_destroy": (ctypes.c_int, [_c_p]),
        "h2_tree_build": (ctypes.c_int, [_c_p, ctypes.c_int, _i64, _c_p, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(_c_p), _c_p]),
        "h2_tree_sizes": (ctypes.c_int, [_c_p, _c_p]),
        "h2_tree_structure": (ctypes.c_int, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
        "h2_compress_kernel": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_c_p)]),
        "h2_compress_kernel_normals": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_int, _c_p,
                                                      ctypes.POINTER(_c_p)]),
        "h2_mul_intermediate": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p, _c_p, ctypes.c_double, ctypes.c_int,
                                               _c_p]),
        "h2_zero_like": (ctypes.c_int, [_c_p, _c_p, ctypes.c_double, ctypes.POINTER(_c_p)]),
        "h2_stats": (ctypes.c_int, [_c_p, ctypes.c_int, ctypes.POINTER(Stats)]),
        "h2_export": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_char_p]),
        "h2_recompress": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p, _c_p, ctypes.c_double, ctypes.c_int]),
        "h2_matvec": (ctypes.c_int, [_c_p, _c_p, ctypes.c_char, ctypes.c_double, _c_p, ctypes.c_double, _c_p,
                                     ctypes.c_int]),
        "h2_matvec_noalloc": (ctypes.c_int, [_c_p, _c_p, ctypes.c_char, ctypes.c_double, _c_p, ctypes.c_double,
                                             _c_p, ctypes.c_int]),
        "h2_product_matvec": (ctypes.c_int, [_c_p, _c_p, ctypes.c_char, ctypes.c_double, _c_p, ctypes.c_double,
                                             _c_p, ctypes.c_int]),
        "h2_to_dense": (ctypes.c_int, [_c_p, _c_p, _c_p, _i64]),
        "h2_product_to_dense": (ctypes.c_int, [_c_p, _c_p, _c_p, _i64]),
        "h2_matrix_basis": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_int, _c_p, _i64]),
        "h2_product_basis": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_int, _c_p, _i64]),
        "h2_matrix_ranks": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p]),
        "h2_product_ranks": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p]),
        "h2_product_sizes": (ctypes.c_int, [_c_p, _c_p]),
        "h2_step_times": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int, ctypes.c_int]),
        "h2_set_rank_rule": (ctypes.c_int, [_c_p, ctypes.c_int]),
        "h2_set_level_factor": (ctypes.c_int, [_c_p, ctypes.c_double]),
        "h2_set_run_scratch": (ctypes.c_int, [_c_p, ctypes.c_int64]),
        "h2_debug_fail_after": (ctypes.c_int, [_c_p, ctypes.c_int]),
        "h2_profile": (ctypes.c_int, [_c_p, ctypes.c_int]),
        "h2_kernel_stats": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p, ctypes.c_int]),
        "h2_tree_destroy": (None, [_c_p]),
        "h2_matrix_destroy": (None, [_c_p]),
        "h2_product_destroy": (None, [_c_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return sig


_lib = None
EXPORTS = None
RANK_RULES = {"abs": 0, "relF": 1}


def load(path: str | None = None):
    """Load libh2.so (raises if it has not been built)."""
    global _lib, EXPORTS
    if path is None and _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_2309_09061_amd.build_lib`")
    lib = ctypes.CDLL(p)
    EXPORTS = _declare(lib)
    if path is None:
        _lib = lib
    return lib


def _check(lib, st):
    if st != 0:
        raise H2Error(st, lib.h2_last_error().decode())


def _ptr(x):
    """Device pointer of a torch tensor, or an integer address."""
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(type(x))


class Context:
    """h2_ctx on a HIP device (device=-1: host-only, symbolic calls only)."""

    def __init__(self, device: int = 0, stream=None, lib=None, allocator="torch"):
        """allocator: "torch" (PyTorch's caching allocator on the context's
        stream), None (the library's own hipMalloc), or a pair of
        (ALLOC_FN, FREE_FN) callbacks."""
        self.lib = lib or load()
        self.h = _c_p()
        if stream is None and device >= 0:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        if device < 0 or allocator is None:
            self._cb = (ALLOC_FN(), FREE_FN())
        elif allocator == "torch":
            self._cb = torch_allocator(device, stream or 0)
        else:
            self._cb = tuple(allocator)
        _check(self.lib, self.lib.h2_ctx_create(device, stream or 0, self._cb[0], self._cb[1], None,
                                                ctypes.byref(self.h)))

    def close(self):
        if self.h:
            _check(self.lib, self.lib.h2_ctx_destroy(self.h))
            self.h = _c_p()

    def set_rank_rule(self, rule: str):
        """Truncation rule of the rank-choosing SVDs: "abs" (singular values
        above eps of the scaled matrices) or "relF" (relative-Frobenius tail
        at most eps)."""
        _check(self.lib, self.lib.h2_set_rank_rule(self.h, RANK_RULES[rule]))

    def set_level_factor(self, zeta: float):
        """Level-dependent tolerances: clusters on level l of a tree of depth
        D truncate at eps * zeta**(D - l) (1: one tolerance on all levels)."""
        _check(self.lib, self.lib.h2_set_level_factor(self.h, float(zeta)))

    def set_run_scratch(self, nbytes: int):
        """Device scratch bound of one run in the steps that take a level in
        runs (<= 0: the default of 4 GiB); lower peak memory, more launches."""
        _check(self.lib, self.lib.h2_set_run_scratch(self.h, int(nbytes)))

    def fail_after(self, launches: int):
        """Test hook: the launches-th batched launch issued by this context's
        own host thread fails before it starts (-1 turns it off)."""
        _check(self.lib, self.lib.h2_debug_fail_after(self.h, launches))

    def profile(self, enable: bool = True, families=None):
        """Time kernel launches with HIP events: every family when `families`
        is None, else only the named ones (names of KERNEL_FAMILIES)."""
        mask = 0
        if enable:
            fams = KERNEL_FAMILIES if families is None else families
            for f in fams:
                mask |= 1 << KERNEL_FAMILIES.index(f)
        _check(self.lib, self.lib.h2_profile(self.h, mask))

    def kernel_stats(self, reset: bool = False) -> dict:
        out = {}
        for kind, name in enumerate(KERNEL_FAMILIES):
            v = np.zeros(4)
            _check(self.lib, self.lib.h2_kernel_stats(self.h, kind, v.ctypes.data, 0))
            out[name] = {"ms": float(v[0]), "launches": int(v[1]), "flops": float(v[2]), "bytes": float(v[3])}
        if reset:
            v = np.zeros(4)
            _check(self.lib, self.lib.h2_kernel_stats(self.h, 0, v.ctypes.data, 1))
        return out

    def step_times(self, host: bool = False, reset: bool = False) -> dict:
        """Device time per step (ms) summed since the last reset; host=True:
        host issue time per step.  Waits for the context's streams."""
        out = np.zeros(16)
        n = self.lib.h2_step_times(self.h, out.ctypes.data, 16, 1 if reset else 0)
        off = 8 if host else 0
        return {STEPS[i]: float(out[off + i]) for i in range(min(8, n - off))}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    def __init__(self, ctx: Context, points: np.ndarray, leaf_size: int, eta: float):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim == 1:
            pts = pts[:, None]
        self.ctx, self.lib = ctx, ctx.lib
        self.n, self.dim = pts.shape
        self.perm = np.zeros(self.n, dtype=np.int64)
        self.h = _c_p()
        _check(self.lib, self.lib.h2_tree_build(ctx.h, self.dim, self.n, pts.ctypes.data, leaf_size, eta,
                                                ctypes.byref(self.h), self.perm.ctypes.data))
        s = np.zeros(7, dtype=np.int64)
        _check(self.lib, self.lib.h2_tree_sizes(self.h, s.ctypes.data))
        self.sizes = dict(zip(["n", "dim", "depth", "nclusters", "nblocks", "nadm", "ninadm"], s.tolist()))

    def structure(self):
        nc, nb = self.sizes["nclusters"], self.sizes["nblocks"]
        off = np.zeros(nc, np.int64)
        size = np.zeros(nc, np.int64)
        br = np.zeros(nb, np.int32)
        bc = np.zeros(nb, np.int32)
        bt = np.zeros(nb, np.int8)
        _check(self.lib, self.lib.h2_tree_structure(self.h, off.ctypes.data, size.ctypes.data, br.ctypes.data,
                                                    bc.ctypes.data, bt.ctypes.data))
        return off, size, br, bc, bt

    def __del__(self):
        try:
            if self.h:
                self.lib.h2_tree_destroy(self.h)
        except Exception:
            pass


class Matrix:
    def __init__(self, ctx: Context, tree: Tree, handle):
        self.ctx, self.lib, self.tree, self.h = ctx, ctx.lib, tree, handle

    @classmethod
    def kernel(cls, ctx: Context, tree: Tree, kernel: str, order: int, normals=None):
        """Chebyshev H^2 approximation of a kernel matrix; normals (n x dim,
        input point order) for the double-layer kernel "dlp"."""
        h = _c_p()
        if normals is None:
            _check(ctx.lib, ctx.lib.h2_compress_kernel(ctx.h, tree.h, KERNELS[kernel], order, ctypes.byref(h)))
        else:
            nrm = np.ascontiguousarray(normals, dtype=np.float64)
            if nrm.shape != (tree.n, tree.dim):
                raise ValueError("normals must be n x dim")
            _check(ctx.lib, ctx.lib.h2_compress_kernel_normals(ctx.h, tree.h, KERNELS[kernel], order,
                                                               nrm.ctypes.data, ctypes.byref(h)))
        return cls(ctx, tree, h)

    @classmethod
    def zero(cls, ctx: Context, tree: Tree, eta: float = 0.0):
        """Z = 0 on the tree's block tree, or on the block tree of
        admissibility parameter eta when eta > 0."""
        h = _c_p()
        _check(ctx.lib, ctx.lib.h2_zero_like(ctx.h, tree.h, eta, ctypes.byref(h)))
        return cls(ctx, tree, h)

    def matvec(self, x, y, alpha=1.0, beta=0.0, op="N"):
        nvec = 1 if len(x.shape) == 1 else x.shape[1]
        _check(self.lib, self.lib.h2_matvec(self.ctx.h, self.h, op.encode(), alpha, _ptr(x), beta, _ptr(y), nvec))

    def matvec_noalloc(self, x, y, alpha=1.0, beta=0.0, op="N"):
        """The same product without any device allocation (fixed scratch)."""
        nvec = 1 if len(x.shape) == 1 else x.shape[1]
        _check(self.lib, self.lib.h2_matvec_noalloc(self.ctx.h, self.h, op.encode(), alpha, _ptr(x), beta,
                                                    _ptr(y), nvec))

    def to_dense(self, out, ld=None):
        _check(self.lib, self.lib.h2_to_dense(self.ctx.h, self.h, _ptr(out), ld or self.tree.n))

    def ranks(self, which=0):
        r = np.zeros(self.tree.sizes["nclusters"], np.int32)
        _check(self.lib, self.lib.h2_matrix_ranks(self.h, which, r.ctypes.data))
        return r

    def basis(self, which, cluster, out, ld):
        _check(self.lib, self.lib.h2_matrix_basis(self.ctx.h, self.h, which, cluster, _ptr(out), ld))

    def __del__(self):
        try:
            if self.h:
                self.lib.h2_matrix_destroy(self.h)
        except Exception:
            pass


class Product:
    def __init__(self, ctx, tree, handle):
        self.ctx, self.lib, self.tree, self.h = ctx, ctx.lib, tree, handle

    def matvec(self, x, y, alpha=1.0, beta=0.0, op="N"):
        nvec = 1 if len(x.shape) == 1 else x.shape[1]
        _check(self.lib, self.lib.h2_product_matvec(self.ctx.h, self.h, op.encode(), alpha, _ptr(x), beta,
                                                    _ptr(y), nvec))

    def to_dense(self, out, ld=None):
        _check(self.lib, self.lib.h2_product_to_dense(self.ctx.h, self.h, _ptr(out), ld or self.tree.n))

    def ranks(self, which=0):
        r = np.zeros(self.tree.sizes["nclusters"], np.int32)
        _check(self.lib, self.lib.h2_product_ranks(self.h, which, r.ctypes.data))
        return r

    def basis(self, which, cluster, out, ld):
        _check(self.lib, self.lib.h2_product_basis(self.ctx.h, self.h, which, cluster, _ptr(out), ld))

    def sizes(self):
        s = np.zeros(5, np.int64)
        _check(self.lib, self.lib.h2_product_sizes(self.h, s.ctypes.data))
        return dict(zip(["nblocks", "nadm", "ninadm", "triples", "bytes"], s.tolist()))

    def __del__(self):
        try:
            if self.h:
                self.lib.h2_product_destroy(self.h)
        except Exception:
            pass


def h2_mul_intermediate(ctx: Context, X, Y, eps: float, precision: str = "fp64"):
    """Phase 1 for one product (X, Y matrices) or for independent products in
    one call (X, Y equal-length lists); returns a Product or a list of them."""
    single = not isinstance(X, (list, tuple))
    xs_l, ys_l = ([X], [Y]) if single else (list(X), list(Y))
    if len(xs_l) != len(ys_l) or not xs_l:
        raise ValueError("X and Y must have the same, non-zero length")
    n = len(xs_l)
    xs = (_c_p * n)(*[x.h for x in xs_l])
    ys = (_c_p * n)(*[y.h for y in ys_l])
    gs = (_c_p * n)()
    _check(ctx.lib, ctx.lib.h2_mul_intermediate(ctx.h, n, ctypes.cast(xs, _c_p), ctypes.cast(ys, _c_p), eps,
                                                PRECISIONS[precision], ctypes.cast(gs, _c_p)))
    out = [Product(ctx, x.tree, _c_p(gs[i])) for i, x in enumerate(xs_l)]
    return out[0] if single else out


def h2_recompress(ctx: Context, G, Z, eps: float, precision: str = "fp64"):
    """Phase 2 for one product or for lists of products and zero targets."""
    single = not isinstance(G, (list, tuple))
    g_l, z_l = ([G], [Z]) if single else (list(G), list(Z))
    if len(g_l) != len(z_l) or not g_l:
        raise ValueError("G and Z must have the same, non-zero length")
    n = len(g_l)
    gs = (_c_p * n)(*[g.h for g in g_l])
    zs = (_c_p * n)(*[z.h for z in z_l])
    _check(ctx.lib, ctx.lib.h2_recompress(ctx.h, n, ctypes.cast(gs, _c_p), ctypes.cast(zs, _c_p), eps,
                                          PRECISIONS[precision]))
    return Z


def h2_tree_build(ctx: Context, points, leaf_size: int, eta: float) -> Tree:
    return Tree(ctx, points, leaf_size, eta)


def h2_compress_kernel(ctx: Context, tree: Tree, kernel: str, order: int) -> Matrix:
    return Matrix.kernel(ctx, tree, kernel, order)


def h2_zero_like(ctx: Context, tree: Tree, eta: float = 0.0) -> Matrix:
    return Matrix.zero(ctx, tree, eta)
