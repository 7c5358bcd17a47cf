"""Seeded synthetic inputs for the Eikonal solvers.

This module only draws problem data (speed arrays, obstacle masks, source
nodes, arrival times); it contains none of the solvers' arithmetic, so both
the GPU path's tests and the CPU oracle consume identical bits from it.

Every generator returns a dict with ``nx, ny, h, F (float64, [ny, nx]),
mask (uint8 [ny, nx] or None), src (int64 linear indices j*nx+i), q (float64)``
plus a ``name``.  The paper's own workloads are analytic speed functions on
the unit square with q = 0 on point or boundary exit sets (Section 4); these
generators follow that recipe with seeded variations (checkerboards with
random per-square speeds, rectangle obstacles, Gaussian bumps, mazes).
"""
from __future__ import annotations

import math

import numpy as np


def _pack(name, F, h, src, q=None, mask=None, **extra):
    ny, nx = F.shape
    src = np.asarray(src, dtype=np.int64).ravel()
    q = np.zeros(len(src)) if q is None else np.asarray(q, dtype=np.float64).ravel()
    d = dict(name=name, nx=nx, ny=ny, h=float(h), F=np.ascontiguousarray(F, dtype=np.float64),
             mask=None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8),
             src=src, q=q)
    d.update(extra)
    return d


def point_source_unit(n: int = 129, lo: float = -1.0, hi: float = 1.0):
    """F = 1 on [lo, hi]^2 with n nodes per side and the source at the centre
    node (n odd).  With n = 129 on [-1, 1]^2 this is h = 1/64, source (64, 64)."""
    h = (hi - lo) / (n - 1)
    F = np.ones((n, n))
    c = (n - 1) // 2
    return _pack(f"const_point_{n}", F, h, [c * n + c], x0=lo)


def smooth_sine(n: int = 1025, amp: float = 0.5, freq: float = 1.0):
    """F(x, y) = 1 + amp sin(2 pi freq x) sin(2 pi freq y) on [0, 1]^2, point
    source at the centre node.  n = 1025, amp = 0.5 is the 1025^2 workload."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    s = np.sin(2.0 * math.pi * freq * x)
    F = 1.0 + amp * np.outer(s, s)
    c = (n - 1) // 2
    return _pack(f"sine_{n}_a{amp}_f{freq}", F, h, [c * n + c])


def sinusoid_point(n: int = 1408, amp: float = 0.5, freq: float = 10.0):
    """F(x, y) = 1 + amp sin(2 pi freq x) sin(2 pi freq y) on [0, 1]^2 with the
    exit set at the centre (0.5, 0.5) (Section 4.3): the centre node with q = 0
    when n is odd, else the four nodes around it with q = their distance to
    the centre."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    s = np.sin(2.0 * math.pi * freq * x)
    F = 1.0 + amp * np.outer(s, s)
    if n % 2:
        c = (n - 1) // 2
        return _pack(f"sine_pt_{n}_a{amp}_f{freq}", F, h, [c * n + c])
    a, b = n // 2 - 1, n // 2
    src = [a * n + a, a * n + b, b * n + a, b * n + b]
    q = [math.hypot(0.5 * h, 0.5 * h)] * 4
    return _pack(f"sine_pt_{n}_a{amp}_f{freq}", F, h, src, q=q)


def checkerboard_point(n: int = 1408, k: int = 11):
    """k x k checkerboard on [0, 1]^2 (checker of node x_i: floor(k x_i)) with
    F = 1 on the slow checkers, the centre one among them, and F = 2 on the
    others; exit set at the centre (0.5, 0.5) as in sinusoid_point
    (Section 4.2)."""
    h = 1.0 / (n - 1)
    idx = np.minimum((np.arange(n) * h * k).astype(np.int64), k - 1)
    parity = (idx[None, :] + idx[:, None]) % 2
    F = np.where(parity == (2 * (k // 2)) % 2, 1.0, 2.0)
    if n % 2:
        c = (n - 1) // 2
        return _pack(f"checker{k}_pt_{n}", F, h, [c * n + c])
    a, b = n // 2 - 1, n // 2
    src = [a * n + a, a * n + b, b * n + a, b * n + b]
    q = [math.hypot(0.5 * h, 0.5 * h) / F[a, a]] * 4
    return _pack(f"checker{k}_pt_{n}", F, h, src, q=q)


def sinusoid_boundary(n: int = 1408, amp: float = 0.5, freq: float = 10.0):
    """F(x, y) = 1 + amp sin(2 pi freq x) sin(2 pi freq y) on [0, 1]^2 with the
    exit set Q = every boundary node, q = 0 (the general boundary conditions
    of Section 4.5)."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    s = np.sin(2.0 * math.pi * freq * x)
    F = 1.0 + amp * np.outer(s, s)
    idx = np.arange(n * n).reshape(n, n)
    src = np.unique(np.concatenate([idx[0], idx[-1], idx[:, 0], idx[:, -1]]))
    return _pack(f"sine_gbc_{n}_a{amp}_f{freq}", F, h, src)


def checker_obstacles(n: int = 4097, squares: int = 16, seed: int = 3, obst_seed: int = 33,
                      cover: float = 0.20, side_lo: int = 64, side_hi: int = 512,
                      keep: int = 16):
    """Piecewise-constant speed on a squares x squares checkerboard with the
    per-square speed ~ U[0.5, 2] (seed), plus axis-aligned rectangular
    obstacles with sides ~ U{side_lo..side_hi} nodes at uniform positions
    (obst_seed), added until they cover >= `cover` of the nodes.  The keep x
    keep block at the source corner (0, 0) stays accessible."""
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(seed)
    Fsq = rng.uniform(0.5, 2.0, size=(squares, squares))
    w = max((n - 1) // squares, 1)
    idx = np.minimum(np.arange(n) // w, squares - 1)
    F = Fsq[np.ix_(idx, idx)]  # [j, i]: row index = y square, column = x square
    mask = np.ones((n, n), dtype=np.uint8)
    orng = np.random.default_rng(obst_seed)
    side_hi = min(side_hi, n)
    side_lo = min(side_lo, side_hi)
    covered = 0
    target = cover * n * n
    while covered < target:
        wx, wy = orng.integers(side_lo, side_hi + 1, size=2)
        x0 = int(orng.integers(0, n - wx + 1))
        y0 = int(orng.integers(0, n - wy + 1))
        mask[y0:y0 + wy, x0:x0 + wx] = 0
        mask[:keep, :keep] = 1
        covered = int(n * n - mask.sum(dtype=np.int64))
    return _pack(f"checker_obst_{n}", F, h, [0], mask=mask,
                 coverage=covered / float(n * n))


def gaussian_bumps(n: int, rng: np.random.Generator, nbumps: int = 4):
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)  # X[j, i] = x_i, Y[j, i] = y_j
    F = np.ones((n, n))
    for _ in range(nbumps):
        A = rng.uniform(-1.0, 1.0)
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        sig = rng.uniform(0.05, 0.3)
        F += A * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    F = np.clip(F, 0.25, 2.0)
    ns = int(rng.integers(1, 5))
    src = rng.choice(n * n, size=ns, replace=False)
    return _pack(f"bumps_{n}", F, h, np.sort(src))


def batch_bumps(count: int = 256, seed: int = 4, n_lo: int = 65, n_hi: int = 1025):
    """`count` independent instances: side ~ U{n_lo..n_hi}, speed = 1 + four
    random Gaussian bumps clipped to [0.25, 2], 1-4 distinct random sources."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(n_lo, n_hi + 1, size=count)
    return [gaussian_bumps(int(n), rng) for n in sides]


def kruskal_maze(n: int, rng: np.random.Generator, w_lo: int = 4, w_hi: int = 16):
    """Maze on an n x n grid: rooms of width w ~ U{w_lo..w_hi} on an m x m
    lattice of pitch w + 2 (2-node walls), passages carved by randomized
    Kruskal over the lattice edges (edges taken in a uniformly random order,
    an edge carved when it joins two components: the minimum spanning tree
    of distinct random edge weights); speed ~ U[0.5, 2] per room and per
    carved passage; one source at a random corridor node."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    w = int(rng.integers(w_lo, w_hi + 1))
    p = w + 2
    m = max((n - 2) // p, 1)
    f_room = rng.uniform(0.5, 2.0, size=(m, m))           # [b, a]: room (a, b)
    # lattice edges: east of room (a, b) for a < m - 1, north of it for b < m - 1
    ea, eb = np.meshgrid(np.arange(m - 1), np.arange(m), indexing="xy")
    na, nb = np.meshgrid(np.arange(m), np.arange(m - 1), indexing="xy")
    u = np.concatenate([(eb * m + ea).ravel(), (nb * m + na).ravel()])
    v = np.concatenate([(eb * m + ea + 1).ravel(), ((nb + 1) * m + na).ravel()])
    ne = (m - 1) * m
    order = rng.permutation(len(u))                        # Kruskal's processing order
    weight = np.empty(len(u))
    weight[order] = np.arange(1, len(u) + 1)
    f_pass = rng.uniform(0.5, 2.0, size=len(u))
    carved = np.zeros(len(u), dtype=bool)
    if len(u):
        T = minimum_spanning_tree(coo_matrix((weight, (u, v)), shape=(m * m, m * m))).tocoo()
        carved[order[(T.data - 1).astype(np.int64)]] = True
    east = np.zeros((m, max(m - 1, 0)), dtype=bool)
    north = np.zeros((max(m - 1, 0), m), dtype=bool)
    east.ravel()[:] = carved[:ne]
    north.ravel()[:] = carved[ne:]
    f_east = f_pass[:ne].reshape(m, max(m - 1, 0))
    f_north = f_pass[ne:].reshape(max(m - 1, 0), m)
    # lattice coordinates of every node row / column
    z = np.arange(n) - 2
    blk, off = z // p, z % p
    inside = (z >= 0) & (blk < m)
    room = inside & (off < w)                              # inside a room's span
    wall = inside & (off >= w) & (blk < m - 1)             # between rooms blk and blk + 1
    bi = np.clip(blk, 0, m - 1)
    bw = np.clip(blk, 0, max(m - 2, 0))
    F = np.ones((n, n))
    mask = np.zeros((n, n), dtype=np.uint8)
    R = room[:, None] & room[None, :]
    F[R] = f_room[bi[:, None], bi[None, :]][R]
    mask[R] = 1
    if m > 1:
        E = room[:, None] & wall[None, :]
        E &= east[bi[:, None], bw[None, :]]
        F[E] = f_east[bi[:, None], bw[None, :]][E]
        mask[E] = 1
        N = wall[:, None] & room[None, :]
        N &= north[bw[:, None], bi[None, :]]
        F[N] = f_north[bw[:, None], bi[None, :]][N]
        mask[N] = 1
    acc = np.flatnonzero(mask.ravel())
    src = int(acc[rng.integers(0, len(acc))])
    h = 1.0 / (n - 1)
    return _pack(f"maze_{n}_w{w}", F, h, [src], mask=mask, corridor=w)


def maze_requests(count: int, seed: int = 5, n_lo: int = 129, n_hi: int = 2049):
    """Serving requests: side n = round(exp(U[ln n_lo, ln n_hi])), a Kruskal
    maze each."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append(kruskal_maze(n, rng))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 5):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed + 1000)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def random_small(rng: np.random.Generator, nx: int, ny: int, obst: float = 0.15,
                 nsrc: int = 2, fmin: float = 0.5, fmax: float = 2.0, q_spread: float = 0.0):
    """Small random problem for cross-checks: random speeds, random obstacle
    nodes, distinct random accessible sources with q ~ U[0, q_spread]."""
    F = rng.uniform(fmin, fmax, size=(ny, nx))
    mask = (rng.uniform(size=(ny, nx)) >= obst).astype(np.uint8)
    acc = np.flatnonzero(mask.ravel())
    if len(acc) == 0:
        mask[0, 0] = 1
        acc = np.array([0])
    src = rng.choice(acc, size=min(nsrc, len(acc)), replace=False)
    q = rng.uniform(0.0, q_spread, size=len(src)) if q_spread > 0 else None
    h = 1.0 / max(nx - 1, 1)
    return _pack(f"rand_{nx}x{ny}", F, h, np.sort(src), q=q, mask=mask)


def config(k: int, **kw):
    """The five workloads the library is measured on (1-based)."""
    if k == 1:
        return point_source_unit(129)
    if k == 2:
        return smooth_sine(1025, 0.5)
    if k == 3:
        return checker_obstacles(4097)
    if k == 4:
        return batch_bumps(**kw)
    if k == 5:
        return maze_requests(kw.pop("count", 64), **kw)
    raise ValueError(k)


# ---------------------------------------------------------------------------
# three dimensions (arrays of shape (nz, ny, nx), node (i, j, k) at
# (k*ny + j)*nx + i)
# ---------------------------------------------------------------------------

def sine3(nx: int, ny: int, nz: int, amp: float = 0.5, freq: float = 1.0):
    """F = 1 + amp sin(2 pi f x) sin(2 pi f y) sin(2 pi f z) on the unit cube
    (h = 1 / (max side - 1)), exit set at the centre node."""
    h = 1.0 / max(max(nx, ny, nz) - 1, 1)
    z, y, x = np.meshgrid(np.arange(nz) * h, np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
    F = 1.0 + amp * np.sin(2 * math.pi * freq * x) * np.sin(2 * math.pi * freq * y) * np.sin(2 * math.pi * freq * z)
    c = ((nz // 2) * ny + ny // 2) * nx + nx // 2
    return dict(name=f"sine3_{nx}x{ny}x{nz}", F=F, h=h, nx=nx, ny=ny, nz=nz,
                src=np.array([c], dtype=np.int64), q=np.array([0.0]), mask=None)


def boxes3(nx: int, ny: int, nz: int, rng: np.random.Generator, nbox: int = 6, nsrc: int = 3):
    """Speed uniform in [0.5, 2] per node, seeded random axis-aligned box
    obstacles, nsrc random exit nodes with costs in [0, 0.2]."""
    h = 1.0 / max(max(nx, ny, nz) - 1, 1)
    F = rng.uniform(0.5, 2.0, size=(nz, ny, nx))
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    for _ in range(nbox):
        a = [int(rng.integers(0, s)) for s in (nz, ny, nx)]
        b = [min(s, a0 + int(rng.integers(1, max(2, s // 3)))) for a0, s in zip(a, (nz, ny, nx))]
        mask[a[0]:b[0], a[1]:b[1], a[2]:b[2]] = 0
    acc = np.flatnonzero(mask.ravel())
    src = rng.choice(acc, size=min(nsrc, len(acc)), replace=False).astype(np.int64)
    q = rng.uniform(0.0, 0.2, size=len(src))
    return dict(name=f"boxes3_{nx}x{ny}x{nz}", F=F, h=h, nx=nx, ny=ny, nz=nz, src=src, q=q, mask=mask)
