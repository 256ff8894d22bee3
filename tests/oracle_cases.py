"""Small cached oracle problems shared by the CPU pin tests."""
import functools

import numpy as np

import oracle as O
import workloads as W

SMALL = {
    # name: (n, dim, leaf, order, kernel_x, kernel_y, eta, seed)
    "1d": (256, 1, 16, 4, "log", "log", 1.0, 1),
    "2d": (512, 2, 32, 3, "log", "expneg", 1.0, 2),
    "2d64": (1024, 2, 64, 4, "log", "expneg", 1.0, 2),
    "sph": (512, 3, 32, 3, "inv4pi", "inv4pi", 2.0, 3),
}


@functools.lru_cache(maxsize=None)
def problem(name):
    n, d, leaf, order, kx, ky, eta, seed = SMALL[name]
    dist = "sphere" if name == "sph" else "uniform"
    pts = W.make_points(seed, n, d, dist)
    tree, bt, X, Y = O.build_problem(pts, leaf, eta, order, kx, ky)
    return pts, tree, bt, X, Y


@functools.lru_cache(maxsize=None)
def dense(name):
    _, _, _, X, Y = problem(name)
    Xd, Yd = X.dense(), Y.dense()
    return Xd, Yd, Xd @ Yd


@functools.lru_cache(maxsize=None)
def product(name, eps):
    _, _, bt, X, Y = problem(name)
    return O.multiply(X, Y, bt, eps)


def rel2(A, B):
    return np.linalg.norm(A - B, 2) / np.linalg.norm(B, 2)


def relF(A, B):
    nb = np.linalg.norm(B)
    return np.linalg.norm(A - B) / (nb if nb > 0 else 1.0)
