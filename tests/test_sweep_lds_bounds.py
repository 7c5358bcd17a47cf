"""LDS index range of the cell sweep (CPU only, no device).

The sweep walks the anti-diagonals of a w x hgt tile held in LDS with pitch
P = S + 2 (one halo row and column on each side); lane l owns column l and
reads the operands of its next step one step ahead.  This test replays the
kernel's index arithmetic for every lane and step -- the lane's row clamped
to the halo rows, lanes past the tile's width on the halo column beside it,
the look-ahead reads east / north / h/F / west of the next position, the
store into the lane's position -- and checks that every LDS access stays
inside the arrays the kernel declares (the tile array has a guard row of P
elements before the tile and 65 elements after it, because on the last
steps the north look-ahead reaches one row past the far halo row; values
read there are never used) and that stores outside the tile's interior land
on its halo, whose h/F the kernel sets to +inf so that those stores write
back the value read."""
import itertools

import pytest


def sweep_indices(S, dirn, w, hgt):
    """(reads of the tile array, reads of the h/F array, writes of the tile
    array) of one sweep, as LDS element indices relative to the tile base."""
    P = S + 2
    sx = 1 if dirn in (0, 1) else -1
    sy = 1 if dirn in (0, 3) else -1
    rowstep = sy * P
    j0 = 0 if sy > 0 else hgt - 1
    nsteps = w + hgt - 1
    reads, dreads, writes = set(), set(), set()
    for lane in range(64):
        col_ok = lane < w
        i = (lane if sx > 0 else w - 1 - lane) if col_ok else (w if sx > 0 else -1)

        def idx_t(t):
            tc = -1 if t < -1 else (hgt if t > hgt else t)
            return (j0 + sy * tc + 1) * P + i + 1

        c, c1 = idx_t(-lane), idx_t(1 - lane)
        reads.add(idx_t(-1))                       # prev
        reads.update((c + sx, c1, c, c - sx))      # first operands
        dreads.add(c)
        for d in range(nsteps):
            t = d - lane
            c2 = c1 + (rowstep if 0 <= t + 2 <= hgt else 0)
            assert c2 == idx_t(t + 2)              # the position two steps on
            reads.update((c1 + sx, c2, c1 - sx))
            dreads.add(c1)
            writes.add(c)
            c, c1 = c1, c2
    return reads, dreads, writes


@pytest.mark.parametrize("S", [16, 32, 64])
def test_sweep_accesses_stay_in_the_lds_arrays(S):
    P = S + 2
    before, size = P, P + P * P + 64 + 1      # the kernel's guarded tile array
    lo, hi = -before, size - before - 1
    shapes = sorted({(w, h) for w in (1, 2, S // 2 + 1, S - 1, S) for h in (1, 2, S // 3 + 1, S - 1, S)})
    touched_guard = False
    for dirn, (w, h) in itertools.product(range(4), shapes):
        reads, dreads, writes = sweep_indices(S, dirn, w, h)
        assert lo <= min(reads) and max(reads) <= hi, (S, dirn, w, h, min(reads), max(reads))
        assert 0 <= min(dreads) and max(dreads) < P * P, (S, dirn, w, h)
        assert 0 <= min(writes) and max(writes) < P * P, (S, dirn, w, h)
        # stores land on the tile with its halo ring (rows 0..h+1, columns
        # 0..w+1) and nowhere else
        for x in writes:
            r, cc = divmod(x, P)
            assert 0 <= r <= h + 1 and 0 <= cc <= w + 1, (S, dirn, w, h, x)
        touched_guard |= min(reads) < 0 or max(reads) > P * P - 1
    # the guards are needed: some full-height sweep reads past the halo rows
    assert touched_guard
