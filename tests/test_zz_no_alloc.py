"""The entry point that allocates nothing (h2_matvec_noalloc) against
h2_matvec on the same inputs, through the C-ABI: two calls in a row, the
second on a smaller matrix, both products of a phase-2 result Z and of an
input kernel matrix; and the refusal of a call beyond the fixed scratch."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def colmajor(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda().t()


def zeros_colmajor(rows, cols):
    return torch.zeros((cols, rows), dtype=torch.float64, device="cuda").t()


def _problem(c, n, leaf, order, seed, eps):
    from paper_2309_09061_amd import h2
    pts = W.make_points(seed, n, 2, "uniform")
    T = h2.Tree(c, pts, leaf, 1.0)
    X = h2.Matrix.kernel(c, T, "log", order)
    Y = h2.Matrix.kernel(c, T, "expneg", order)
    G = h2.h2_mul_intermediate(c, X, Y, eps)
    Z = h2.h2_recompress(c, G, h2.Matrix.zero(c, T), eps)
    return T, X, Z


def test_noalloc_matvec_matches_matvec():
    from paper_2309_09061_amd import h2
    h2.load()
    c = h2.Context(0)
    for n, leaf, order, nvec, seed, op, beta in ((16384, 64, 4, 6, 21, "N", 0.0), (3000, 32, 3, 2, 22, "T", 0.5)):
        _say(f"[gpu] noalloc matvec: n={n} nvec={nvec} op={op}")
        T, X, Z = _problem(c, n, leaf, order, seed, 1e-6)
        x = colmajor(W.probe_vectors(seed + 100, n, nvec))
        y0 = colmajor(W.probe_vectors(seed + 200, n, nvec))
        for A in (Z, X):
            ref = y0.clone()
            got = y0.clone()
            A.matvec(x, ref, alpha=1.5, beta=beta, op=op)
            A.matvec_noalloc(x, got, alpha=1.5, beta=beta, op=op)
            torch.cuda.synchronize()
            r, g = ref.cpu().numpy(), got.cpu().numpy()
            # the same kernels in the same order: equal to the last bit
            assert np.array_equal(r, g), float(np.abs(r - g).max())


def test_noalloc_matvec_refuses_beyond_scratch():
    from paper_2309_09061_amd import h2
    h2.load()
    c = h2.Context(0)
    n = 16384
    T, X, _ = _problem(c, n, 64, 4, 23, 1e-6)
    nvec = 600  # the result alone needs n * nvec * 8 bytes = 78.6 MB > 64 MiB
    x = zeros_colmajor(n, nvec)
    y = torch.full((nvec, n), 7.0, dtype=torch.float64, device="cuda").t()
    with pytest.raises(h2.H2Error) as e:
        X.matvec_noalloc(x, y)
    assert e.value.code == 1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())  # untouched
    # the context stays usable, and a call that fits works afterwards
    x = colmajor(W.probe_vectors(24, n, 3))
    ref, got = zeros_colmajor(n, 3), zeros_colmajor(n, 3)
    X.matvec(x, ref)
    X.matvec_noalloc(x, got)
    torch.cuda.synchronize()
    assert np.array_equal(ref.cpu().numpy(), got.cpu().numpy())
