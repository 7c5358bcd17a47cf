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


# --------------------------------------------------------------------------
# Fast Marching-Sweeping in three dimensions (Algorithm FMSM on cells of
# s^3 nodes, readings of the coarse speed and the sweep choice as in two
# dimensions)
# --------------------------------------------------------------------------

def test_fmsm3_orderings_per_axis():
    """Sweep choice per axis (codes: bit 0 x descending, bit 1 y descending,
    bit 2 z descending; faces: bit 2 axis + side, side 1 = high face)."""
    def codes(m):
        return {d for d in range(8) if m >> d & 1}
    assert codes(O.fmsm3_orderings(0)) == set(range(8))  # no earlier neighbour: all
    assert codes(O.fmsm3_orderings(0b111111)) == set(range(8))
    assert codes(O.fmsm3_orderings(0b000001)) == {0, 2, 4, 6}  # low x: x ascending
    assert codes(O.fmsm3_orderings(0b000010)) == {1, 3, 5, 7}  # high x: x descending
    assert codes(O.fmsm3_orderings(0b011001)) == {2}  # low x, high y, low z
    assert codes(O.fmsm3_orderings(0b100110)) == {5}  # high x, low y, high z
    assert codes(O.fmsm3_orderings(0b000101)) == {0, 4}  # low x, low y; z free
    assert codes(O.fmsm3_orderings(0b000101, 0b100)) == {0}  # ... one node thick in z
    assert codes(O.fmsm3_orderings(0, 0b100)) == {0, 1, 2, 3}


def slab(F, h, src, q=None, mask=None):
    return O.Problem3(F[None], h, src, q, None if mask is None else mask[None])


@pytest.mark.parametrize("case", range(4))
def test_fmsm3_slab_equals_two_dimensional_fmsm(case):
    """nz = 1: 3-D FMSM is the (paper-pinned) 2-D FMSM bit for bit: same
    coarse order, same sweeps, same values (sides chosen so that the 2-D
    tiling merges no one-node cell)."""
    from paper_1110_6220_amd import workloads as W
    rng = np.random.default_rng(40 + case)
    if case == 0:
        w = W.sinusoid_point(94, 0.5, 3.0)
    elif case == 1:
        w = W.checkerboard_point(118, 11)
    elif case == 2:
        w = W.random_small(rng, 77, 59, obst=0.15, nsrc=3, q_spread=0.2)
    else:
        w = W.sinusoid_boundary(70, 0.99, 1.0)
    for s in (8, 5):
        p2 = O.Problem.from_workload(w)
        V2, st2 = O.fmsm(p2, s)
        V3, st3 = O.fmsm3(slab(w["F"], w["h"], w["src"], w.get("q"), w.get("mask")), s)
        assert np.array_equal(V2, V3[0], equal_nan=False), (case, s)
        assert st2["sweeps"] == st3["sweeps"] and st2["cells"] == st3["cells"]
        assert np.array_equal(st2["order"], st3["order"])


def test_fmsm3_constant_speed_is_exact():
    """F constant, one exit node: every cell's characteristics leave its
    earlier-accepted faces, so the chosen sweeps reach Fast Marching's values."""
    for n, s, c in [((33, 33, 33), 8, (16, 16, 16)), ((29, 21, 40), 8, (3, 17, 30)),
                    ((24, 24, 24), 6, (0, 0, 0))]:
        F = np.full(n[::-1], 1.7)
        p = O.Problem3(F, 0.05, [idx(n, *c)])
        U = O.fmm3(p)
        V, st = O.fmsm3(p, s)
        assert np.abs(V - U).max() <= 1e-15 * U.max(), (n, s)
        assert 1.0 <= st["sweeps"] / st["cells"] < 3.0


@pytest.mark.parametrize("seed", range(3))
def test_fmsm3_bounds_the_exact_solution(seed):
    """FMSM's values are upper bounds of the discrete solution (only finitely
    many updates from values that are themselves upper bounds), equal on the
    exit nodes, infinite where it is (and possibly also behind obstacles that
    a cell's one-pass directional sweeps cannot go around)."""
    rng = np.random.default_rng(seed)
    p = random_problem(rng, (19, 23, 17))
    U = O.fmm3(p)
    for s in (4, 8):
        V, _ = O.fmsm3(p, s)
        fin = np.isfinite(U)
        assert (V[fin] >= U[fin] * (1 - 1e-15)).all()
        assert not np.isfinite(V[~fin]).any()
        assert np.array_equal(V.ravel()[p.src], U.ravel()[p.src])


def test_fmsm3_error_shrinks_with_smaller_cells():
    """On a smooth speed FMSM's additional error falls as the cells shrink
    (toward one node per cell, where FMSM sweeps every node from its
    accepted neighbours)."""
    from paper_1110_6220_amd import workloads as W
    p = O.Problem3.from_workload(W.sine3(41, 41, 41, 0.5, 1.0))
    U = O.fmm3(p)
    errs = [np.abs(O.fmsm3(p, s)[0] - U).max() for s in (10, 5, 2)]
    assert errs[0] > errs[1] > errs[2] >= 0.0


@pytest.mark.parametrize("s", [5, 7])
def test_fmsm3_part_one_is_fast_marching_on_cell_centres(s):
    """Part I: with an odd cell side the coarse speed is F at the centre node
    of each cell (the last cells ragged), so the coarse values are the
    (pinned) 3-D Fast Marching on those samples with h^c = s h, and the cell
    order is its acceptance order."""
    from paper_1110_6220_amd import workloads as W
    w = W.sine3(4 * s + 3, 3 * s + 1, 2 * s + 5, 0.6, 1.5)
    p = O.Problem3.from_workload(w)
    _, st = O.fmsm3(p, s)
    centre = [None] * 3
    for a, m in enumerate((p.nx, p.ny, p.nz)):
        lo = np.arange(0, m, s)
        hi = np.minimum(lo + s, m)
        centre[a] = (lo + hi - 1) // 2  # centre node of [lo, hi) (the lower one when even)
    Fc = w["F"][np.ix_(centre[2], centre[1], centre[0])]
    K = (len(centre[0]), len(centre[1]), len(centre[2]))
    src_cell = []
    for x in w["src"]:
        i, j, k = x % p.nx, (x // p.nx) % p.ny, x // (p.nx * p.ny)
        src_cell.append(((k // s) * K[1] + j // s) * K[0] + i // s)
    cp = O.Problem3(Fc, s * p.h, src_cell)
    Uc, order = O.fmm3(cp, want_order=True)
    ragged = [a for a in range(3) if (p.nx, p.ny, p.nz)[a] % s % 2 == 0 and (p.nx, p.ny, p.nz)[a] % s]
    assert not ragged  # the sizes above give odd extents in every cell
    assert np.array_equal(st["coarse_u"], Uc)
    assert np.array_equal(st["order"][: len(order)], order)
