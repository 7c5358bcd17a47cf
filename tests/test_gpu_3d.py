"""GPU parity of the 3-D exact solver (eik_solve3) against the 3-D oracle's
Fast Marching: FP64 within 1e-12 relative with identical sets of infinite
nodes, on cells with ragged edges, obstacles with unreachable pockets,
several exit nodes, an exit set covering the boundary, and degenerate
shapes."""
import numpy as np
import pytest

import oracle as O
from paper_1110_6220_amd import workloads as W
from gpu_util import max_rel

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def eik():
    import torch
    assert torch.cuda.is_available()
    from paper_1110_6220_amd import eik as E
    return E


def dev(w):
    import torch
    d = torch.device("cuda:0")
    return (torch.from_numpy(w["F"]).to(d), torch.from_numpy(w["src"]).to(d),
            torch.from_numpy(w["q"]).to(d),
            None if w.get("mask") is None else torch.from_numpy(w["mask"]).to(d))


def boundary_exit(n):
    w = W.sine3(n, n, n, 0.4, 1.0)
    k, j, i = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    on = (i == 0) | (j == 0) | (k == 0) | (i == n - 1) | (j == n - 1) | (k == n - 1)
    w["src"] = np.flatnonzero(on.ravel()).astype(np.int64)
    w["q"] = np.zeros(len(w["src"]))
    return w


def cases():
    rng = np.random.default_rng(21)
    return [W.sine3(33, 33, 33, 0.0), W.sine3(41, 37, 29, 0.5), W.boxes3(40, 24, 17, rng),
            W.boxes3(27, 30, 33, np.random.default_rng(5), nbox=10, nsrc=1), boundary_exit(25),
            W.sine3(64, 64, 16, 0.5), W.sine3(1, 1, 1), W.sine3(2, 2, 70), W.sine3(50, 30, 1)]


@pytest.mark.parametrize("case", range(10))
def test_exact_3d_matches_fast_marching(eik, case):
    w = (cases() + [fmsm_special()])[case]
    U = O.fmm3(O.Problem3.from_workload(w))
    F, src, q, mask = dev(w)
    print(f"[gpu] 3-D {w['name']}", flush=True)
    u, st = eik.eik_solve3(F, w["h"], src, q, mask)
    got = u.cpu().numpy()
    assert max_rel(got, U) <= TOL64
    s = np.asarray(w["src"])
    assert (got.ravel()[s] == U.ravel()[s]).all()  # exit nodes keep q exactly
    assert st["rounds"] >= 1 and st["cell_visits"] >= 1


def test_host_inputs_match_device_inputs(eik):
    w = W.boxes3(30, 20, 25, np.random.default_rng(8))
    print("[gpu] 3-D host vs device", flush=True)
    uh, _ = eik.eik_solve3(w["F"], w["h"], w["src"], w["q"], w["mask"])
    F, src, q, mask = dev(w)
    ud, _ = eik.eik_solve3(F, w["h"], src, q, mask)
    assert max_rel(uh, ud.cpu().numpy()) <= TOL64


def test_device_validation(eik):
    """Device inputs are validated on the device: a non-positive speed or a
    source on an obstacle is EINVAL."""
    w = W.boxes3(20, 20, 20, np.random.default_rng(2))
    F, src, q, mask = dev(w)
    F[3, 4, 5] = -1.0
    print("[gpu] 3-D device validation", flush=True)
    with pytest.raises(eik.EikError) as e:
        eik.eik_solve3(F, w["h"], src, q, None)
    assert e.value.code == eik.EIK_EINVAL


def test_device_pointers_must_be_aligned(eik):
    """A device u_out off 8-byte alignment is EINVAL, rejected on the host
    before any launch (the kernels update u with 64-bit atomics)."""
    import torch
    w = W.sine3(9, 9, 9, 0.0)
    F, src, q, _ = dev(w)
    buf = torch.empty(F.numel() + 1, dtype=torch.float64, device=F.device)
    print("[gpu] 3-D misaligned u_out", flush=True)
    rc = eik.lib.eik_solve3(9, 9, 9, float(w["h"]), F.data_ptr(), None, src.numel(), src.data_ptr(),
                            q.data_ptr(), buf.data_ptr() + 4, 1, eik._stream_of(True), None)
    assert rc == eik.EIK_EINVAL
    assert b"aligned" in eik.lib.eik_last_error()


# --------------------------------------------------------------------------
# FMSM in three dimensions: bitwise equal to the oracle's 3-D FMSM (same
# coarse order, same orderings, same directional update), cells of 8^3 nodes
# --------------------------------------------------------------------------

def fmsm_special():
    """Coarse obstacles (an 8-node wall on a cell layer sealing x >= 32),
    unreached accessible cells behind it, and cells whose centre nodes are
    all obstacles (their coarse speed falls back to the cell mean)."""
    nx, ny, nz = 41, 27, 19
    h = 1.0 / (max(nx, ny, nz) - 1)
    z, y, x = np.meshgrid(np.arange(nz) * h, np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
    F = 1.0 + 0.6 * np.sin(5.0 * x) * np.cos(4.0 * y) * np.sin(3.0 * z + 0.5)
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    mask[:, :, 24:32] = 0                 # the wall: cells with cx = 3 are all obstacles
    mask[3:5, 3:5, 3:5] = 0               # centre nodes of cell (0, 0, 0)
    mask[11:13, 11:13, 11:13] = 0         # centre nodes of cell (1, 1, 1)
    c = (9 * ny + 20) * nx + 13
    return dict(name="fmsm_special", F=F, h=h, nx=nx, ny=ny, nz=nz, src=np.array([c], dtype=np.int64),
                q=np.array([0.0]), mask=mask)


def fmsm_cases():
    rng = np.random.default_rng(33)
    return [W.sine3(33, 33, 33, 0.5), W.sine3(41, 37, 29, 0.9, 1.5), W.sine3(33, 33, 33, 0.0),
            W.boxes3(40, 24, 17, rng), W.boxes3(27, 30, 33, np.random.default_rng(5), nbox=10, nsrc=1),
            boundary_exit(25), W.sine3(64, 64, 16, 0.5), W.sine3(1, 1, 1), W.sine3(2, 2, 70),
            W.sine3(50, 30, 1, 0.7, 2.0), fmsm_special()]


@pytest.mark.parametrize("case", range(11))
def test_fmsm3_matches_oracle_bitwise(eik, case):
    w = fmsm_cases()[case]
    V, st_o = O.fmsm3(O.Problem3.from_workload(w), 8)
    F, src, q, mask = dev(w)
    print(f"[gpu] 3-D FMSM {w['name']}", flush=True)
    u, st = eik.eik_solve3(F, w["h"], src, q, mask, method="fmsm")
    got = u.cpu().numpy()
    assert np.array_equal(got, V)
    assert st["sweeps"] == st_o["sweeps"] and st["cell_visits"] == st_o["removals"]


def test_fmsm3_host_inputs_match_device_inputs(eik):
    w = W.boxes3(30, 20, 25, np.random.default_rng(9))
    print("[gpu] 3-D FMSM host vs device", flush=True)
    uh, _ = eik.eik_solve3(w["F"], w["h"], w["src"], w["q"], w["mask"], method="fmsm")
    F, src, q, mask = dev(w)
    ud, _ = eik.eik_solve3(F, w["h"], src, q, mask, method="fmsm")
    assert np.array_equal(uh, ud.cpu().numpy())


def test_fmsm3_coarse_grid_in_device_memory(eik):
    """More coarse cells (20^3 = 8000) than the LDS-resident coarse Fast
    Marching holds: the variant with its state in device memory, still
    bitwise equal to the oracle."""
    w = W.sine3(160, 160, 160, 0.5)
    V, st_o = O.fmsm3(O.Problem3.from_workload(w), 8)
    F, src, q, mask = dev(w)
    print("[gpu] 3-D FMSM 160^3", flush=True)
    u, st = eik.eik_solve3(F, w["h"], src, q, mask, method="fmsm")
    assert np.array_equal(u.cpu().numpy(), V)
    assert st["sweeps"] == st_o["sweeps"]
