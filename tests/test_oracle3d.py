"""Pins of the 3-D oracle (the extension of the methods to three dimensions:
six neighbours, the three-sided upwind update).  The paper prints no 3-D
values, so the pins are closed forms and independent methods: plane fronts
along an axis, a face diagonal and the space diagonal are reproduced exactly;
a one-node-thick slab equals the (paper-pinned) 2-D oracle bit for bit; Fast
Marching equals brute-force value iteration and Fast Sweeping on random
small problems with obstacles; acceptance is monotone; the fixed-point
residual vanishes; a point source converges to the Euclidean distance."""
import math

import numpy as np
import pytest

import oracle as O

INF = math.inf


def idx(n, i, j, k):
    nx, ny, nz = n
    return (k * ny + j) * nx + i


def test_update_closed_forms():
    ulp = 2.0 ** -52
    for d in (0.1, 1.0, 3.7):
        for a in (0.0, 0.25, 5.0):
            assert O.update3(a, INF, INF, d) == a + d
            assert abs(O.update3(a, a, INF, d) - (a + d / math.sqrt(2))) <= 4 * ulp * (a + d)
            assert abs(O.update3(a, a, a, d) - (a + d / math.sqrt(3))) <= 4 * ulp * (a + d)
        # one-sided when the gap is at least delta, in any argument order
        assert O.update3(INF, 2.0 + d, 2.0, d) == 2.0 + d
    assert O.update3(INF, INF, INF, 1.0) == INF
    rng = np.random.default_rng(1)
    for _ in range(2000):  # with no third neighbour: the 2-D update, bit for bit
        a, b, d = rng.uniform(0, 2), rng.uniform(0, 2), rng.uniform(0.01, 1)
        assert O.update3(a, b, INF, d) == O.update(a, b, d)
        assert O.update3(INF, a, b, d) == O.update(a, b, d)


def plane_wave(n, normal, F=1.0):
    """Exit set = the faces the front enters through, with q the exact
    arrival time of the plane front u = (normal . x) / F (normal a unit
    vector of non-negative entries)."""
    nx, ny, nz = n
    h = 1.0 / 16
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    exact = (normal[0] * i + normal[1] * j + normal[2] * k) * h / F
    face = np.zeros(n[::-1], bool)
    if normal[0] > 0: face[:, :, 0] = True
    if normal[1] > 0: face[:, 0, :] = True
    if normal[2] > 0: face[0, :, :] = True
    src = np.flatnonzero(face.ravel())
    p = O.Problem3(np.full(n[::-1], F), h, src, exact.ravel()[src])
    return p, exact


@pytest.mark.parametrize("normal", [(1, 0, 0), (0, 0, 1), (1 / math.sqrt(2), 1 / math.sqrt(2), 0),
                                    (1 / math.sqrt(3), 1 / math.sqrt(3), 1 / math.sqrt(3))])
def test_plane_fronts_exact(normal):
    """Linear solutions solve the discrete equations exactly: a front along
    an axis (one-sided updates), a face diagonal (two-sided) and the space
    diagonal (three-sided)."""
    p, exact = plane_wave((9, 8, 7), normal, F=1.3)
    V = O.fmm3(p)
    assert np.abs(V - exact).max() <= 1e-14 * exact.max()
    W, _ = O.fsm3(p)
    assert np.abs(W - exact).max() <= 1e-14 * exact.max()


def random_problem(rng, n):
    nx, ny, nz = n
    F = rng.uniform(0.5, 2.0, size=(nz, ny, nx))
    mask = (rng.uniform(size=(nz, ny, nx)) > 0.15).astype(np.uint8)
    acc = np.flatnonzero(mask.ravel())
    src = rng.choice(acc, size=int(rng.integers(1, 4)), replace=False)
    q = rng.uniform(0, 0.3, size=len(src))
    return O.Problem3(F, 0.1, src, q, mask)


def rel(a, b):
    fin = np.isfinite(b)
    assert np.array_equal(np.isfinite(a), fin)
    return float((np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)).max())


def test_fmm_equals_value_iteration_and_sweeping():
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = tuple(int(x) for x in rng.integers(3, 8, size=3))
        p = random_problem(rng, n)
        V, order = O.fmm3(p, want_order=True)
        J, _ = O.jacobi3(p)
        W, _ = O.fsm3(p)
        assert rel(V, J) <= 1e-13 and rel(V, W) <= 1e-13
        vals = V.ravel()[order[len(np.unique(p.src)):]]
        assert (np.diff(vals) >= -1e-15 * np.maximum(vals[1:], 1.0)).all()  # monotone acceptance


def test_slab_equals_two_dimensional_oracle():
    """nz = 1: the 3-D methods on a slab are the 2-D methods bit for bit."""
    rng = np.random.default_rng(3)
    F = rng.uniform(0.5, 2.0, size=(23, 31))
    mask = (rng.uniform(size=F.shape) > 0.1).astype(np.uint8)
    src = np.flatnonzero(mask.ravel())[[5, 300]]
    q = np.array([0.0, 0.05])
    V2 = O.fmm(O.Problem(F, 0.05, src, q, mask))
    V3 = O.fmm3(O.Problem3(F[None], 0.05, src, q, mask[None]))
    assert np.array_equal(V2, V3[0])


def test_residual_and_distance_convergence():
    errs = []
    for n in (9, 17, 33):
        c = n // 2
        p = O.Problem3(np.ones((n, n, n)), 1.0 / (n - 1), [idx((n, n, n), c, c, c)])
        V = O.fmm3(p)
        assert O.residual3(p, V)[0] <= 1e-13
        g = np.arange(n) * p.h - 0.5
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        errs.append(np.abs(V - np.sqrt(x * x + y * y + z * z)).max())
    assert errs[0] > errs[1] > errs[2]
    order = math.log2(errs[1] / errs[2])
    assert 0.5 <= order <= 1.1, (errs, order)
