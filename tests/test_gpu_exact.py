"""GPU parity of the exact (label-correcting on cells) method against the CPU
oracle's Fast Marching solution: FP64 within 1e-12 relative with identical
+inf patterns, on seeded inputs covering several tiles, ragged tails,
obstacles, unreachable pockets, multiple sources and degenerate grids."""
import numpy as np
import pytest

import gpu_util
import oracle as O
from gpu_util import max_rel, to_dev
from paper_1110_6220_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def eik():
    import torch
    assert torch.cuda.is_available()
    from paper_1110_6220_amd import eik as E
    return E


def solve_dev(eik, w, **kw):
    return gpu_util.solve_dev(eik, w, **kw)


def test_constant_speed_point_source(eik):
    w = W.config(1)
    U = O.fmm(O.Problem.from_workload(w))
    for cell in (16, 8, 32, 64):
        got, st = solve_dev(eik, w, cell=cell)
        assert max_rel(got, U) <= TOL64, cell
        assert st["cells"] > 0 and st["cell_visits"] >= st["cells"]


@pytest.mark.parametrize("seed", range(6))
def test_random_problems_with_obstacles(eik, seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(4):
        nx, ny = (int(v) for v in rng.integers(5, 150, size=2))
        w = W.random_small(rng, nx, ny, obst=float(rng.uniform(0.0, 0.3)),
                           nsrc=int(rng.integers(1, 5)), q_spread=float(rng.choice([0.0, 0.5])))
        U = O.fmm(O.Problem.from_workload(w))
        for cell in (4, 8, 16, 32, 64):
            got, _ = solve_dev(eik, w, cell=cell)
            assert max_rel(got, U) <= TOL64, (nx, ny, cell)


def test_ragged_tiles_and_degenerate_grids(eik):
    rng = np.random.default_rng(7)
    cases = [(1, 1, [0]), (1, 37, [5]), (37, 1, [36]), (2, 2, [3]), (65, 65, [0]),
             (66, 130, [66 * 64 + 3]), (129, 17, [0, 128, 129 * 16])]
    for nx, ny, src in cases:
        F = rng.uniform(0.5, 2.0, size=(ny, nx))
        w = W._pack(f"deg_{nx}x{ny}", F, 0.1, src)
        U = O.fmm(O.Problem.from_workload(w))
        for cell in (4, 16, 64):
            got, _ = solve_dev(eik, w, cell=cell)
            assert max_rel(got, U) <= TOL64, (nx, ny, cell)


@pytest.mark.parametrize("n,cell", [(769, 64), (289, 32), (129, 16), (65, 64), (1025, 32)])
def test_last_cell_one_node_wider(eik, n, cell):
    """n = 1 (mod s): the standard tiling would merge a one-node last cell into
    a cell wider than the tile; every node must still be solved."""
    w = W.smooth_sine(n, 0.4, 2.0)
    w["src"] = np.array([0, n * n - 1, (n // 3) * n + n // 2], dtype=np.int64)
    w["q"] = np.zeros(3)
    U = O.fmm(O.Problem.from_workload(w))
    got, st = solve_dev(eik, w, cell=cell)
    assert max_rel(got, U) <= TOL64
    assert st["cell_used"] == cell


def test_every_node_a_source(eik):
    F = np.ones((20, 30))
    w = W._pack("allsrc", F, 0.1, np.arange(600), q=np.linspace(0.0, 1.0, 600))
    got, _ = solve_dev(eik, w, cell=8)
    assert np.array_equal(got.ravel(), np.linspace(0.0, 1.0, 600))


def test_smooth_speed_1025_fp64(eik):
    """The 1025^2 smooth-speed workload at every cell side."""
    w = W.config(2)
    U = O.fmm(O.Problem.from_workload(w))
    for cell in (64, 32, 16, 8):
        got, st = solve_dev(eik, w, cell=cell)
        err = max_rel(got, U)
        print(f"  cell {cell}: max rel {err:.2e}, AvHR {st['AvHR']:.3f}, AvS {st['AvS']:.3f}, "
              f"kernel {st['kernel_seconds']*1e6:.0f} us", flush=True)
        assert err <= TOL64


def test_host_pointers_match_device_pointers(eik):
    rng = np.random.default_rng(3)
    w = W.random_small(rng, 90, 70, obst=0.2, nsrc=3, q_spread=0.2)
    got_dev, _ = solve_dev(eik, w, cell=16)
    got_host, _ = eik.eik_solve(w["F"], w["h"], w["src"], w["q"], w["mask"], cell=16)
    assert np.array_equal(got_dev, got_host)


def test_device_validation_leaves_output_untouched(eik):
    import torch
    w = W.random_small(np.random.default_rng(5), 40, 40, obst=0.1, nsrc=1)
    d = to_dev(w)
    d["F"][3, 3] = -1.0
    if "mask" in d:
        d["mask"][3, 3] = 1
    u = torch.full_like(d["F"], 42.0)
    with pytest.raises(eik.EikError) as ex:
        eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"), u_out=u)
    assert ex.value.code == eik.EIK_EINVAL
    assert bool((u == 42.0).all())
    d = to_dev(w)
    with pytest.raises(eik.EikError):
        eik.eik_solve(d["F"], d["h"], torch.tensor([40 * 40], device="cuda:0"), u_out=u)
    assert bool((u == 42.0).all())


def test_device_exit_nodes_out_of_range(eik):
    """Device exit-node indices far outside the grid (negative, or beyond
    2^31 nodes) are EINVAL for every method that orders cells on the coarse
    grid, and no kernel maps them to a cell."""
    import torch
    w = W.random_small(np.random.default_rng(7), 40, 40, obst=0.0, nsrc=1)
    d = to_dev(w)
    u = torch.full_like(d["F"], 42.0)
    for method in ("exact", "hcm", "fmsm"):
        for bad in (-1, -100000, 2 ** 40, -(2 ** 40)):
            print(f"[gpu] {method} exit node {bad}", flush=True)
            src = torch.tensor([0, bad], dtype=torch.int64, device="cuda:0")
            with pytest.raises(eik.EikError) as ex:
                eik.eik_solve(d["F"], d["h"], src, u_out=u, method=method, cell=8)
            assert ex.value.code == eik.EIK_EINVAL
            assert bool((u == 42.0).all())


def test_device_pointers_must_be_aligned(eik):
    """Device u_out off its element alignment is EINVAL for the cell solver
    and the whole-grid sweep, rejected on the host before any launch."""
    import ctypes
    import torch
    w = W.random_small(np.random.default_rng(6), 20, 20, obst=0.0, nsrc=1)
    d = to_dev(w)
    buf = torch.empty(20 * 20 + 1, dtype=torch.float64, device="cuda:0")
    o = eik._opts(eik.F64, "exact", 0, 0.0, True, eik._stream_of(True), False, 0, 0, 0, False,
                  "auto", 0, False)
    print("[gpu] misaligned u_out", flush=True)
    rc = eik.lib.eik_solve(20, 20, float(d["h"]), d["F"].data_ptr(), None, d["src"].numel(),
                           d["src"].data_ptr(), d["q"].data_ptr(), buf.data_ptr() + 4,
                           ctypes.byref(o), None)
    assert rc == eik.EIK_EINVAL and b"aligned" in eik.lib.eik_last_error()
    so = eik.SweepOpts(eik.F64, 0, 0, 0.0, 1, eik._stream_of(True))
    rc = eik.lib.eik_sweep_solve(20, 20, float(d["h"]), d["F"].data_ptr(), None, d["src"].numel(),
                                 d["src"].data_ptr(), d["q"].data_ptr(), buf.data_ptr() + 4,
                                 ctypes.byref(so), None, None, None)
    assert rc == eik.EIK_EINVAL and b"aligned" in eik.lib.eik_last_error()


def test_fp32_within_bound(eik):
    """FP32 storage with the FP64 two-sided branch: max and L1 error against
    the FP64 oracle stay within D * 2^-24 * u_max (D = longest dependency
    chain, bounded by the number of nodes on a monotone path, nx + ny)."""
    for w in (W.config(1), W.smooth_sine(257)):
        U = O.fmm(O.Problem.from_workload(w))
        got, _ = solve_dev(eik, w, cell=32, dtype="f32")
        fin = np.isfinite(U)
        err = np.abs(got[fin] - U[fin])
        D = w["nx"] + w["ny"]
        bound = D * 2.0 ** -24 * U[fin].max()
        print(f"  fp32 {w['name']}: max {err.max():.2e} L1 {err.sum() * w['h'] ** 2:.2e} "
              f"bound {bound:.2e}", flush=True)
        assert err.max() <= bound


def test_time_limit_is_reported(eik):
    """A solve stopped by its time limit fails with EDEVICE instead of
    returning a partial result (the limit is forced from the host: workers
    give up between cells, every kernel exits normally)."""
    w = W.config(2)
    d = to_dev(w)
    print("[gpu] 1025^2 solve with a 1 ms limit", flush=True)
    with pytest.raises(eik.EikError) as e:
        eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, timeout_ms=1, cell=16)
    assert e.value.code == eik.EIK_EDEVICE
    got, _ = solve_dev(eik, w)  # the next solve is unaffected
    assert max_rel(got, O.fmm(O.Problem.from_workload(w))) <= TOL64


def test_probe_step_latency(eik):
    """The sweep-step latency probe (the t_dep of the span bound) returns a
    positive time of the order of one dependent FP64 update (tens to
    hundreds of nanoseconds), and rejects what it does not measure."""
    for dt in ("f64", "f32"):
        for side in (32, 64):
            t = eik.probe_step_latency(dt, side, 50)
            print(f"  t_dep {dt} side {side}: {t * 1e9:.1f} ns", flush=True)
            assert 5e-9 < t < 5e-6
    with pytest.raises(eik.EikError):
        eik.probe_step_latency("f64", 16, 10)
