"""Seeded synthetic workloads for adaptive H^2-matrix multiplication.

This module only generates inputs: point sets, kernel identifiers and the
parameters of each workload.  It holds none of the method's arithmetic and is
the one module that both the FP64 oracle (``oracle/``) and the HIP path
(``paper_2309_09061_amd``) are fed from.

The paper measures on Galerkin boundary-element matrices compressed by hybrid
cross approximation (Section 7); those meshes and matrices are not available,
so every workload here is a point-collocation kernel matrix on seeded random
points with the kernel, manifold, size and tolerance of the paper's
single-layer experiment or of a smaller analogue.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Kernel identifiers shared with the C-ABI (include/h2.h, enum h2_kernel).
KERNELS = {
    "log": 0,       # log|x-y|, diagonal 0
    "expneg": 1,    # exp(-|x-y|), diagonal 1
    "inv4pi": 2,    # 1/(4 pi |x-y|), diagonal 0 (single-layer kernel, Section 7)
    "inv": 3,       # 1/|x-y|, diagonal 0
    "dlp": 4,       # <n(x), x-y> / (4 pi |x-y|^3), diagonal 0 (double-layer kernel, Section 7)
    "poly2": 100,   # (x.y)^2: a polynomial of degree 2, reproduced exactly by order >= 3
}


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    n: int
    dim: int
    distribution: str          # "uniform" (unit cube) or "sphere" (normalised Gaussians)
    leaf_size: int
    eta: float
    order: int                 # Chebyshev points per axis; rank k = order**dim
    kernel_x: str
    kernel_y: str
    eps: float
    note: str = ""

    @property
    def rank(self) -> int:
        return self.order ** self.dim

    def points(self) -> np.ndarray:
        return make_points(self.seed, self.n, self.dim, self.distribution)

    def normals(self):
        """Unit normals at the points (input order) where the points lie on a
        surface with a kernel that uses them; else None."""
        if self.distribution == "cube_surface":
            return cube_surface_normals(self.points())
        return None


def make_points(seed: int, n: int, dim: int, distribution: str) -> np.ndarray:
    """n x dim float64 points, row-major, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    if distribution == "uniform":
        return np.ascontiguousarray(rng.random((n, dim)), dtype=np.float64)
    if distribution == "sphere":
        g = rng.standard_normal((n, dim))
        return np.ascontiguousarray(g / np.linalg.norm(g, axis=1, keepdims=True))
    if distribution == "cube_surface":
        # uniform on the surface of [-1, 1]^3: a face (axis, sign) per point,
        # uniform coordinates in (-1, 1) on the other two axes
        if dim != 3:
            raise ValueError("cube_surface points are 3-D")
        face = rng.integers(0, 6, n)
        pts = rng.uniform(-1.0, 1.0, (n, 3))
        ax, sign = face // 2, np.where(face % 2 == 0, -1.0, 1.0)
        pts[np.arange(n), ax] = sign
        return np.ascontiguousarray(pts)
    raise ValueError(f"unknown distribution {distribution!r}")


def cube_surface_normals(points: np.ndarray) -> np.ndarray:
    """Outward unit normals of points on the surface of [-1, 1]^3 (input
    order): the axis whose coordinate is exactly -1 or 1, with its sign."""
    ax = np.argmax(np.abs(points), axis=1)
    nrm = np.zeros_like(points)
    nrm[np.arange(points.shape[0]), ax] = np.sign(points[np.arange(points.shape[0]), ax])
    return nrm


# The five workloads.  "c1" is the small case the oracle finishes in seconds;
# "c2" is the single-GPU workload the benchmark is quoted on.
C1 = Workload("c1_1d_log_n1024", 1, 1024, 1, "uniform", 16, 1.0, 4, "log", "log", 1e-8,
              "1-D, X = Y, plain FP64")
C2 = Workload("c2_2d_log_expneg_n16384", 2, 16384, 2, "uniform", 64, 1.0, 4, "log", "expneg", 1e-6,
              "2-D, X log|x-y|, Y exp(-|x-y|), FP64 vs FP32 bulk")
C3 = Workload("c3_sphere_slp_n131072", 3, 131072, 3, "sphere", 64, 2.0, 3, "inv4pi", "inv4pi", 1e-4,
              "unit sphere, single-layer kernel, X = Y")
C5 = Workload("c5_cube_inv_n1048576", 5, 1 << 20, 3, "uniform", 128, 2.0, 4, "inv", "inv", 1e-5,
              "unit cube volume, X = Y")

# The double-layer workload of the paper's second experiment (Section 7):
# the surface of [-1, 1]^3 with the double-layer kernel (not symmetric),
# n = 110592, one of the paper's sizes for it; X = Y.
C6 = Workload("dlp_cube_n110592", 60, 110592, 3, "cube_surface", 64, 2.0, 3, "dlp", "dlp", 1e-4,
              "cube surface, double-layer kernel, X = Y (not symmetric)")

# The same recipe at n = 49152 (another of the paper's sizes): the size at
# which the oracle's results are stored for parity at many levels.
C6S = Workload("dlp_cube_n49152", 61, 49152, 3, "cube_surface", 64, 2.0, 3, "dlp", "dlp", 1e-4,
               "cube surface, double-layer kernel, X = Y (not symmetric)")

# The recipe of c5 at n = 16384 (leaf 128, order 4: k = 64): the size at which
# the oracle's results are stored for parity, with G's ranks up to 165.
C5S = Workload("c5_cube_inv_n16384", 5, 16384, 3, "uniform", 128, 2.0, 4, "inv", "inv", 1e-5,
               "unit cube volume, X = Y, k = 64")

# The same recipe at n = 2^17, the bench's large cube case (no stored
# oracle results: its error is reported against X Y).
C5M = Workload("c5_cube_inv_n131072", 5, 1 << 17, 3, "uniform", 128, 2.0, 4, "inv", "inv", 1e-5,
               "unit cube volume, X = Y, k = 64")

WORKLOADS = {w.name: w for w in (C1, C2, C3, C5, C5M, C5S, C6, C6S)}


def batched_instances(count: int = 64):
    """The 64 independent 2-D products of the batched workload.

    Instance i draws n_i log-uniformly in [2048, 32768] and the order m_i
    uniformly from {3, 4, 5} with default_rng(4000 + i); points are then drawn
    from the same generator.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(4000 + i)
        n_i = int(round(math.exp(rng.uniform(math.log(2048), math.log(32768)))))
        m_i = int(rng.integers(3, 6))
        pts = np.ascontiguousarray(rng.random((n_i, 2)), dtype=np.float64)
        w = Workload(f"c4_inst{i}", 4000 + i, n_i, 2, "uniform", 64, 1.0, m_i, "log", "log", 1e-6)
        out.append((w, pts))
    return out


def small(name: str, n: int, dim: int, leaf: int, order: int, kx: str, ky: str, eps: float,
          eta: float = 1.0, seed: int = 7, distribution: str = "uniform") -> Workload:
    """A reduced workload for tests (same recipe, smaller n)."""
    return Workload(name, seed, n, dim, distribution, leaf, eta, order, kx, ky, eps)


def probe_vectors(seed: int, n: int, count: int) -> np.ndarray:
    """Gaussian probe vectors (n x count, column-major friendly) for matrix comparisons."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, count)))
