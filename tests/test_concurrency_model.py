"""CPU model of the GPU's concurrent cell processing (no device).

The exact method processes cells concurrently: persistent workers pop queued
cells, load the cell with its one-node halo, sweep it until a sweep changes
nothing or leaves no node below an upwind neighbour inside the cell (the
back-flow stop rule that replaces the confirming sweep), publish the
boundary, re-queue neighbours by the add criterion of Algorithm
generic_LC_cells with "changed" meaning strictly decreased since this
processing loaded the cell (reading C11), and store the cell.  A cell
re-requested while it runs is processed again by the same worker with a
fresh halo.  The Theorem of Section 3.2.1 says any removal order reaches the
solution of eq. Eik_discr; what it does not cover is the GPU's concurrency:
halo values read while neighbours are being written.

This model replays that protocol step by step under random interleavings of
several workers.  A halo read returns any value the node held between the
moment the reader popped its cell (every write published before that is
visible, by the queue's release/acquire pairing) and now -- a random mix of
old and new values, as concurrently running neighbours produce.  The final
values must equal the oracle's Fast Marching solution on random problems
with obstacles, several exit nodes and ragged cells."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_6220_amd import workloads as W

INF = math.inf


def update(a, b, dl):
    lo = min(a, b)
    if lo == INF:
        return INF
    d = a - b
    if abs(d) >= dl:
        return lo + dl
    return 0.5 * (a + b + math.sqrt(2.0 * dl * dl - d * d))


def fmsm_dirs(sides):
    """First-sweep choice: corners between inflow sides (0 W, 1 E, 2 S, 3 N)."""
    W_, E_, S_, N_ = (bool(sides >> k & 1) for k in range(4))
    d = 0
    if (W_ or E_) and (S_ or N_):
        d |= (S_ and W_) << 0 | (N_ and W_) << 1 | (N_ and E_) << 2 | (S_ and E_) << 3
    else:
        d |= (3 if W_ else 0) | (12 if E_ else 0) | (9 if S_ else 0) | (6 if N_ else 0)
    return d


class Model:
    def __init__(self, w, s, workers, rng):
        self.nx, self.ny = w["nx"], w["ny"]
        self.rng = rng
        n = self.nx * self.ny
        mask = np.ones(n, bool) if w.get("mask") is None else w["mask"].ravel().astype(bool)
        F = w["F"].ravel()
        self.delta = [w["h"] / F[k] if mask[k] else INF for k in range(n)]
        self.u = [INF] * n
        self.hist = [[(0, INF)] for _ in range(n)]  # (event time, value) per node
        self.clock = 0
        for k, q in zip(w["src"], w["q"]):
            k = int(k)
            self.write(k, min(self.u[k], float(q)))
            self.delta[k] = INF  # exit nodes are frozen
        self.src = {int(k) for k in w["src"]}
        self.s = s
        self.kx, self.ky = -(-self.nx // s), -(-self.ny // s)
        J = self.kx * self.ky
        self.pending = [False] * J
        self.running = [False] * J
        self.flags = [0] * J
        self.sides = [0] * J
        self.visits = [0] * J
        self.queue = []
        for k in self.src:
            self.request(self.cell_of(k), 0, 0)
        self.workers = [None] * workers

    def write(self, k, v):
        self.clock += 1
        self.u[k] = v
        self.hist[k].append((self.clock, v))

    def stale_read(self, k, since):
        """Any value node k held between time `since` and now."""
        h = self.hist[k]
        first = max(i for i, (t, _) in enumerate(h) if t <= since) if h[0][0] <= since else 0
        return h[int(self.rng.integers(first, len(h)))][1]

    def cell_of(self, k):
        return (k // self.nx) // self.s * self.kx + (k % self.nx) // self.s

    def box(self, c):
        cx, cy = c % self.kx, c // self.kx
        return (cx * self.s, min((cx + 1) * self.s, self.nx), cy * self.s, min((cy + 1) * self.s, self.ny))

    def request(self, c, dirs, side_bits):
        self.flags[c] |= dirs
        self.sides[c] |= side_bits
        if not self.pending[c] and not self.running[c]:
            self.queue.append(c)
        self.pending[c] = True

    # one worker's processing of a cell, as a generator of interleaving points
    def process(self, c):
        while True:
            self.pending[c] = False
            self.running[c] = True
            self.visits[c] += 1
            fl, sides = self.flags[c], self.sides[c]
            self.flags[c] = self.sides[c] = 0
            t_pop = self.clock
            yield
            x0, x1, y0, y1 = self.box(c)
            tile = {}
            for j in range(y0 - 1, y1 + 1):
                for i in range(x0 - 1, x1 + 1):
                    inside = x0 <= i < x1 and y0 <= j < y1
                    corner = (i in (x0 - 1, x1)) and (j in (y0 - 1, y1))
                    if corner:
                        continue
                    if not (0 <= i < self.nx and 0 <= j < self.ny):
                        tile[i, j] = INF
                    elif inside:
                        tile[i, j] = self.u[j * self.nx + i]  # only this worker writes it
                    else:
                        tile[i, j] = self.stale_read(j * self.nx + i, t_pop)
            start = dict(tile)
            yield
            # sweeps: first from a corner between inflow sides (else a flagged
            # direction), then reverse the axis with back-flow, until converged
            lead = fmsm_dirs(sides)
            pick = lead or fl
            d = (pick & -pick).bit_length() - 1 if pick else 0
            flip_x = True
            for k in range(64):
                res = self.sweep(tile, x0, x1, y0, y1, d)
                if not (res & 6):
                    break
                if k >= 7:
                    d = (k + 1) & 3
                elif (res & 6) == 6:
                    d ^= 3 if flip_x else 1
                    flip_x = not flip_x
                elif res & 2:
                    d ^= 3
                    flip_x = False
                else:
                    d ^= 1
                    flip_x = True
            else:
                raise AssertionError("cell sweeps did not terminate")
            yield
            # publish: boundary values first, then the add criterion
            first = self.visits[c] == 1
            for (i, j), v in tile.items():
                if x0 <= i < x1 and y0 <= j < y1 and v < start[i, j]:
                    self.write(j * self.nx + i, v)
            nbrs = []
            for side, (di, dj) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
                cx, cy = c % self.kx + di, c // self.kx + dj
                if not (0 <= cx < self.kx and 0 <= cy < self.ky):
                    continue
                if side <= 1:
                    i = x0 if side == 0 else x1 - 1
                    line = [(i, j) for j in range(y0, y1)]
                else:
                    j = y0 if side == 2 else y1 - 1
                    line = [(i, j) for i in range(x0, x1)]
                crit = False
                for (i, j) in line:
                    v, across = tile[i, j], tile[i + di, j + dj]
                    k_in, k_out = j * self.nx + i, (j + dj) * self.nx + i + di
                    changed = v < start[i, j] or (first and k_in in self.src)
                    if changed and self.delta[k_out] != INF and v < across:
                        crit = True
                if crit:
                    recv = side ^ 1
                    nbrs.append((cy * self.kx + cx, (3, 12, 9, 6)[recv], 1 << recv))
            yield
            for nb, dirs, sb in nbrs:
                self.request(nb, dirs, sb)
            yield
            self.running[c] = False
            if not self.pending[c]:
                return
            if c in self.queue:
                self.queue.remove(c)  # re-requested while running: again at once

    def sweep(self, tile, x0, x1, y0, y1, d):
        sx = 1 if d in (0, 1) else -1
        sy = 1 if d in (0, 3) else -1
        xs = range(x0, x1) if sx > 0 else range(x1 - 1, x0 - 1, -1)
        ys = range(y0, y1) if sy > 0 else range(y1 - 1, y0 - 1, -1)
        changed = back_x = back_y = False
        for ii, i in enumerate(xs):
            for jj, j in enumerate(ys):
                dl = self.delta[j * self.nx + i]
                if dl == INF:
                    continue
                a = min(tile[i - 1, j], tile[i + 1, j])
                b = min(tile[i, j - 1], tile[i, j + 1])
                r = min(tile[i, j], update(a, b, dl))
                if r < tile[i, j]:
                    tile[i, j] = r
                    changed = True
                    back_x |= ii > 0 and r < tile[i - sx, j]
                    back_y |= jj > 0 and r < tile[i, j - sy]
        return changed | back_x << 1 | back_y << 2

    def run(self):
        live = {}
        while self.queue or live:
            free = [k for k in range(len(self.workers)) if k not in live]
            if self.queue and free and (not live or self.rng.random() < 0.5):
                c = self.queue.pop(int(self.rng.integers(len(self.queue))))
                live[free[0]] = self.process(c)
            k = list(live)[int(self.rng.integers(len(live)))]
            try:
                next(live[k])
            except StopIteration:
                del live[k]
        return np.array(self.u).reshape(self.ny, self.nx)


@pytest.mark.parametrize("seed", range(8))
def test_concurrent_cells_reach_the_discrete_solution(seed):
    rng = np.random.default_rng(100 + seed)
    nx, ny = (int(v) for v in rng.integers(14, 34, size=2))
    w = W.random_small(rng, nx, ny, obst=0.15, nsrc=int(rng.integers(1, 4)), q_spread=0.3)
    U = O.fmm(O.Problem.from_workload(w))
    for s, workers in ((4, 4), (5, 3), (7, 6)):
        got = Model(w, s, workers, rng).run()
        fin = np.isfinite(U)
        assert np.array_equal(np.isfinite(got), fin), (seed, s)
        rel = np.abs(got[fin] - U[fin]) / np.maximum(U[fin], 1e-300)
        assert rel.max() <= 1e-12, (seed, s, rel.max())


def test_stale_reads_occur():
    """The interleavings do produce halo reads older than the newest value."""
    rng = np.random.default_rng(7)
    w = W.random_small(rng, 30, 26, obst=0.1, nsrc=2)
    m = Model(w, 4, 6, rng)
    stale = [0]
    orig = m.stale_read

    def counting(k, since):
        v = orig(k, since)
        stale[0] += v > m.u[k]
        return v
    m.stale_read = counting
    m.run()
    assert stale[0] > 0


class OneSweep(Model):
    """Planted mistake: a visit stops after its first sweep, whatever the
    back-flow test says."""
    def sweep(self, *a):
        return super().sweep(*a) & 1


class NoRequeue(Model):
    """Planted mistake: a cell is queued only for its first processing."""
    def request(self, c, dirs, side_bits):
        if self.visits[c] == 0:
            super().request(c, dirs, side_bits)


class OldHalo(Model):
    """Planted mistake: halo reads may return values older than the ones
    published before the cell was popped (no acquire ordering)."""
    def stale_read(self, k, since):
        return super().stale_read(k, 0)


@pytest.mark.parametrize("mutant", [OneSweep, NoRequeue, OldHalo])
def test_model_rejects_planted_mistakes(mutant):
    """The model has teeth: each planted mistake misses the solution on
    some of these problems."""
    bad = 0
    for seed in range(8):
        rng = np.random.default_rng(300 + seed)
        w = W.random_small(rng, 24, 22, obst=0.1, nsrc=2)
        U = O.fmm(O.Problem.from_workload(w))
        got = mutant(w, 4, 4, rng).run()
        fin = np.isfinite(U)
        bad += (not np.array_equal(np.isfinite(got), fin)) or \
            np.abs(got[fin] - U[fin]).max() > 1e-12 * U[fin].max()
    assert bad > 0
