"""Index arithmetic of the 3-D round kernel, replayed on the CPU (no device).

For every cell of the grids the 3-D GPU tests use, and every lane of the
wave that processes it, this test recomputes the addresses the round kernel
forms -- the loads of the (8 + 2)^3-node block around the cell and of h/F of
the cell, the LDS indices of the sweep's seven operands on every
anti-diagonal plane of every ordering, the write-back of decreased nodes,
the face scan of the add criterion (including the node across each face and
its h/F), and the neighbour cell queued -- and checks each one against the
bounds of the array it indexes.  The cell count of a round is at most the
number of cells (a cell is listed once per round), so list slots stay in
range as well."""
import itertools

import pytest

C3 = 8
P3 = C3 + 2
SHAPES = [(33, 33, 33), (41, 37, 29), (40, 24, 17), (27, 30, 33), (25, 25, 25), (64, 64, 16),
          (1, 1, 1), (2, 2, 70), (50, 30, 1), (30, 20, 25), (20, 20, 20), (9, 9, 9), (160, 160, 160)]


def cell_lo3(c, n):
    return c * C3 if c * C3 < n else n


def check_cell(nx, ny, nz, cx, cy, cz):
    kx, ky, kz = (-(-n // C3) for n in (nx, ny, nz))
    n = nx * ny * nz
    sxy = nx * ny
    x0, y0, z0 = cx * C3, cy * C3, cz * C3
    w, hg, dp = cell_lo3(cx + 1, nx) - x0, cell_lo3(cy + 1, ny) - y0, cell_lo3(cz + 1, nz) - z0
    assert 1 <= w <= C3 and 1 <= hg <= C3 and 1 <= dp <= C3
    NT, ND = -(-P3 ** 3 // 64), C3 ** 3 // 64
    for lane in range(64):
        for r in range(NT):                      # block of u with halo
            t = lane + 64 * r
            a, b, e = t % P3 - 1, (t // P3) % P3 - 1, t // (P3 * P3) - 1
            i, j, k = x0 + a, y0 + b, z0 + e
            inside = (t < P3 ** 3 and a <= w and b <= hg and e <= dp and i >= 0 and j >= 0 and
                      k >= 0 and i < nx and j < ny and k < nz)
            if inside:
                assert 0 <= k * sxy + j * nx + i < n
            if t < P3 ** 3:
                assert 0 <= t < P3 ** 3
        for r in range(ND):                      # h/F of the cell, write-back
            t = lane + 64 * r
            a, b, e = t % C3, (t // C3) % C3, t // (C3 * C3)
            if a < w and b < hg and e < dp:
                assert 0 <= (z0 + e) * sxy + (y0 + b) * nx + x0 + a < n
                assert 0 <= ((e + 1) * P3 + b + 1) * P3 + a + 1 < P3 ** 3
            assert t < C3 ** 3
    for dirn in range(8):                        # sweeps over anti-diagonal planes
        sx, sy, sz = (-1 if dirn & 1 else 1), (-1 if dirn & 2 else 1), (-1 if dirn & 4 else 1)
        for lane in range(64):
            ii, jj = lane % C3, lane // C3
            i = ii if sx > 0 else w - 1 - ii
            j = jj if sy > 0 else hg - 1 - jj
            col = ii < w and jj < hg
            for d in range(w + hg + dp - 2):
                kk = d - ii - jj
                if not (col and 0 <= kk < dp):
                    continue
                k = kk if sz > 0 else dp - 1 - kk
                t = ((k + 1) * P3 + j + 1) * P3 + i + 1
                ci = (k * C3 + j) * C3 + i
                for o in (0, 1, -1, P3, -P3, P3 * P3, -P3 * P3):
                    assert 0 <= t + o < P3 ** 3
                assert 0 <= ci < C3 ** 3
    for f in range(6):                           # add criterion on the faces
        ax, side = f >> 1, f & 1
        has = [(cx + 1 < kx) if side else cx > 0, (cy + 1 < ky) if side else cy > 0,
               (cz + 1 < kz) if side else cz > 0][ax]
        if not has:
            continue
        n0 = hg if ax == 0 else w
        n1 = hg if ax == 2 else dp
        lim = (w, hg, dp)[ax]
        pos, across = (lim - 1, lim) if side else (0, -1)
        for t in range(n0 * n1):
            p0, p1 = t % n0, t // n0
            if ax == 0:
                a, b, e, aa, bb, ee = pos, p0, p1, across, p0, p1
            elif ax == 1:
                a, b, e, aa, bb, ee = p0, pos, p1, p0, across, p1
            else:
                a, b, e, aa, bb, ee = p0, p1, pos, p0, p1, across
            assert 0 <= (e * C3 + b) * C3 + a < C3 ** 3
            assert 0 <= ((e + 1) * P3 + b + 1) * P3 + a + 1 < P3 ** 3
            assert 0 <= ((ee + 1) * P3 + bb + 1) * P3 + aa + 1 < P3 ** 3
            gi, gj, gk = x0 + aa, y0 + bb, z0 + ee
            assert 0 <= gi < nx and 0 <= gj < ny and 0 <= gk < nz
        c = (cz * ky + cy) * kx + cx
        nb = c + (1 if side else -1) * (1, kx, kx * ky)[ax]
        assert 0 <= nb < kx * ky * kz


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_round_kernel_indices_in_bounds(shape):
    nx, ny, nz = shape
    kx, ky, kz = (-(-n // C3) for n in shape)
    cells = list(itertools.product(range(kx), range(ky), range(kz)))
    if len(cells) > 300:  # large grids: the boundary cells and a sample of the interior
        edge = [c for c in cells if 0 in c or c[0] == kx - 1 or c[1] == ky - 1 or c[2] == kz - 1]
        cells = edge[::7] + cells[::97]
    for cx, cy, cz in cells:
        check_cell(nx, ny, nz, cx, cy, cz)
