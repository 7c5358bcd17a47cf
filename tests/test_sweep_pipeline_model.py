"""Data flow of the cell sweep's anti-diagonal wavefront (CPU only, no device).

The kernel's sweep keeps each lane's operands in registers and reads them
one step ahead: the upwind x value arrives from the lane to the left, the
upwind y value is the lane's own previous result, a lane's row is clamped to
the halo rows before and after its column's turn, lanes past the tile's
width walk the halo column beside the tile, and every lane stores its
result each step with no select, which is correct because the halo's h/F
is +inf in LDS (the update then leaves the value read).  This test replays
that data flow lane by lane with numpy and checks that one sweep leaves the
tile bit for bit as a plain serial Gauss-Seidel sweep in the same order
(Algorithm FSM's lexicographic order for that direction), with the same
decrease and back-flow bits, for ragged tiles, every direction, the
quadrant update and FMSM's sweep-directional one.  Both sides use the same
scalar update (the test is about the order of the data, not its
arithmetic)."""
import itertools

import numpy as np
import pytest

INF = np.inf


def vmin(x, y):
    """IEEE minNum, as v_min_f64: a NaN operand yields the other one."""
    return np.where(np.isnan(x), y, np.where(np.isnan(y), x, np.minimum(x, y)))


def update(a, b, dl):
    with np.errstate(invalid="ignore", over="ignore"):
        lo = vmin(a, b)
        d = a - b
        one = lo + dl
        two = 0.5 * ((a + b) + np.sqrt(2.0 * dl * dl - d * d))
        return np.where(np.abs(d) >= dl, one, two)


def pipeline_sweep(tu_mem, td, kb, P, w, hgt, dirn, directional, mistake=False):
    """The kernel's data flow; tu_mem holds the tile at offset kb.
    mistake: read the next north value one row past the lane's next position
    even where the row is clamped (a planted error)."""
    sx = 1 if dirn in (0, 1) else -1
    sy = 1 if dirn in (0, 3) else -1
    rowstep = sy * P
    j0 = 0 if sy > 0 else hgt - 1
    lanes = np.arange(64)
    col_ok = lanes < w
    i = np.where(col_ok, np.where(sx > 0, lanes, w - 1 - lanes), w if sx > 0 else -1)

    def idx_t(t):
        return (j0 + sy * np.clip(t, -1, hgt) + 1) * P + i + 1

    U = lambda idx: tu_mem[kb + idx]
    c, c1 = idx_t(-lanes), idx_t(1 - lanes)
    prev = U(idx_t(-1 + 0 * lanes))
    ev, nv, uo, dl, hw = U(c + sx), U(c + rowstep if mistake else c1), U(c), td[c], U(c - sx)
    m_dec, m_bx, m_by = np.zeros(64, bool), np.zeros(64, bool), np.zeros(64, bool)
    for d in range(w + hgt - 1):
        t = d - lanes
        c2 = c1 + np.where((t + 2 >= 0) & (t + 2 <= hgt), rowstep, 0)
        evn, nvn, dln, hwn = U(c1 + sx), U(c1 + rowstep if mistake else c2), td[c1], U(c1 - sx)
        wv = np.concatenate(([hw[0]], prev[:-1]))      # DPP wave_shr:1, lane 0 gets hw
        a = wv if directional else vmin(wv, ev)
        b = prev if directional else vmin(prev, nv)
        r = vmin(uo, update(a, b, dl))
        dec = (r < uo) & (t >= 0) & (t < hgt) & col_ok
        m_dec |= dec
        m_bx |= dec & (r < wv)
        m_by |= dec & (r < prev) & (t > 0)
        tu_mem[kb + c] = r                            # every lane stores
        prev = r
        c, c1 = c1, c2
        ev, uo, nv, dl, hw = evn, nv, nvn, dln, hwn
    return bool(m_dec.any()), bool(m_bx[1:].any()), bool(m_by.any())


def serial_sweep(tile, dt, w, hgt, dirn, directional):
    """Plain Gauss-Seidel in the sweep's lexicographic order on a
    (hgt + 2) x (w + 2) array with halo."""
    sx = 1 if dirn in (0, 1) else -1
    sy = 1 if dirn in (0, 3) else -1
    ch = bx = by = False
    for jj in range(hgt):
        y = jj if sy > 0 else hgt - 1 - jj
        for ii in range(w):
            x = ii if sx > 0 else w - 1 - ii
            Y, X = y + 1, x + 1
            up_x, up_y = tile[Y, X - sx], tile[Y - sy, X]
            if directional:
                a, b = up_x, up_y
            else:
                a = vmin(tile[Y, X - 1], tile[Y, X + 1])
                b = vmin(tile[Y - 1, X], tile[Y + 1, X])
            uo = tile[Y, X]
            r = vmin(uo, update(np.float64(a), np.float64(b), dt[Y, X]))
            if r < uo:
                ch = True
                bx |= ii > 0 and r < up_x
                by |= jj > 0 and r < up_y
            tile[Y, X] = r
    return ch, bx, by


def random_tile(rng, w, hgt):
    """Values with a front: a few small exit-like values, +inf patches,
    obstacles (h/F = +inf) and a random halo."""
    tile = np.full((hgt + 2, w + 2), INF)
    tile[1:-1, 1:-1] = np.where(rng.random((hgt, w)) < 0.5, INF, rng.random((hgt, w)) * 5)
    for side in range(4):
        vals = np.where(rng.random(max(w, hgt) + 2) < 0.3, INF, rng.random(max(w, hgt) + 2) * 3)
        if side == 0:
            tile[1:-1, 0] = vals[:hgt]
        elif side == 1:
            tile[1:-1, -1] = vals[:hgt]
        elif side == 2:
            tile[0, 1:-1] = vals[:w]
        else:
            tile[-1, 1:-1] = vals[:w]
    dt = np.where(rng.random((hgt + 2, w + 2)) < 0.1, INF, 0.05 + rng.random((hgt + 2, w + 2)) * 0.2)
    return tile, dt


@pytest.mark.parametrize("S", [16, 32])
def test_wavefront_equals_serial_sweep(S):
    P = S + 2
    kb = P                                             # guard row before the tile
    rng = np.random.default_rng(S)
    shapes = [(w, h) for w in (1, 2, S // 2 + 1, S) for h in (1, 3, S - 1, S)]
    for (w, h), dirn, directional in itertools.product(shapes, range(4), (False, True)):
        tile, dt = random_tile(rng, w, h)
        # LDS image: the tile at pitch P, stale values elsewhere; the halo's
        # h/F is +inf, as after halo_to_masks
        tu_mem = np.full(P + P * P + 65, 7.0)
        td = np.full(P * P, 0.3)
        for Y in range(h + 2):
            tu_mem[kb + Y * P: kb + Y * P + w + 2] = tile[Y]
            td[Y * P: Y * P + w + 2] = dt[Y]
        td_sweep = td.copy()
        for Y in range(h + 2):
            for X in range(w + 2):
                if Y in (0, h + 1) or X in (0, w + 1):
                    td_sweep[Y * P + X] = INF
        bits = pipeline_sweep(tu_mem, td_sweep, kb, P, w, h, dirn, directional)
        ref = tile.copy()
        ref_bits = serial_sweep(ref, dt, w, h, dirn, directional)
        got = np.array([tu_mem[kb + Y * P: kb + Y * P + w + 2] for Y in range(h + 2)])
        assert np.array_equal(got[1:-1, 1:-1], ref[1:-1, 1:-1]), (S, w, h, dirn, directional)
        assert np.array_equal(got, ref), ("halo changed", S, w, h, dirn, directional)
        assert bits == ref_bits, (S, w, h, dirn, directional, bits, ref_bits)


def test_a_planted_carry_mistake_is_caught():
    """Carrying the north value read for the lane's previous position as the
    next step's own value even while the row is clamped (so that a lane's
    first row sees its own old value instead of the halo below) must break
    the equality with the serial sweep."""
    S, w, h = 16, 16, 16
    P, kb = S + 2, S + 2
    rng = np.random.default_rng(5)
    caught = 0
    for dirn, directional in itertools.product(range(4), (False, True)):
        tile, dt = random_tile(rng, w, h)
        tile[1:-1, 1:-1] = INF
        tile[0, 1:-1] = tile[-1, 1:-1] = 0.1            # low halo rows
        tu_mem = np.full(P + P * P + 65, 7.0)
        td = np.full(P * P, INF)
        for Y in range(1, h + 1):
            tu_mem[kb + Y * P: kb + Y * P + w + 2] = tile[Y]
            td[Y * P + 1: Y * P + w + 1] = dt[Y, 1:-1]
        for Y in (0, h + 1):
            tu_mem[kb + Y * P: kb + Y * P + w + 2] = tile[Y]
        pipeline_sweep(tu_mem, td, kb, P, w, h, dirn, directional, mistake=True)
        ref = tile.copy()
        serial_sweep(ref, np.where(np.isfinite(dt), dt, dt), w, h, dirn, directional)
        got = np.array([tu_mem[kb + Y * P: kb + Y * P + w + 2] for Y in range(h + 2)])
        caught += not np.array_equal(got[1:-1, 1:-1], ref[1:-1, 1:-1])
    assert caught == 8
