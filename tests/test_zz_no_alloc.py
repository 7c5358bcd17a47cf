"""eik_solve_noalloc (the allocation-free entry point) against eik_solve,
through the C ABI: two calls in a row, the second on a smaller grid, each
compared with eik_solve on the same inputs (exact method: within 1e-12
relative with identical infinite sets; FMSM: bit for bit).  Also the limits
it states: device pointers only, and a grid beyond its scratch is refused
before any device work."""
import ctypes

import numpy as np
import pytest

import gpu_util
from paper_1110_6220_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eik():
    import torch
    assert torch.cuda.is_available()
    from paper_1110_6220_amd import eik as E
    return E


def noalloc(eik, w, dtype="f64", method="exact", cell=0, u=None):
    import torch
    d = gpu_util.to_dev(w, dtype)
    if u is None:
        u = torch.empty_like(d["F"])
    mask = d.get("mask")
    o = eik._opts(eik.F64 if dtype == "f64" else eik.F32, method, cell, 0.0, True,
                  eik._stream_of(True), False, 0, 0)
    st = eik.Stats()
    print(f"[gpu] eik_solve_noalloc {w['name']} {w['nx']}x{w['ny']} {dtype} {method}", flush=True)
    rc = eik.lib.eik_solve_noalloc(w["nx"], w["ny"], w["h"], d["F"].data_ptr(),
                                   None if mask is None else mask.data_ptr(), d["src"].numel(),
                                   d["src"].data_ptr(), d["q"].data_ptr(), u.data_ptr(),
                                   ctypes.byref(o), ctypes.byref(st))
    torch.cuda.synchronize()
    return rc, u.double().cpu().numpy(), st.as_dict()


def test_two_calls_match_eik_solve(eik):
    rng = np.random.default_rng(5)
    big = W.checker_obstacles(1025, seed=3, obst_seed=33)
    small = W.random_small(rng, 77, 53, obst=0.15, nsrc=3)
    for w in (big, small):
        rc, got, st = noalloc(eik, w)
        assert rc == eik.EIK_OK, eik.last_error()
        ref, _ = gpu_util.solve_dev(eik, w)
        assert gpu_util.max_rel(got, ref) <= 1e-12
        assert st["cells"] > 0 and st["cell_visits"] >= st["cells"]
    for w in (W.smooth_sine(513), W.config(1)):
        for dtype in ("f64", "f32"):
            rc, got, _ = noalloc(eik, w, dtype=dtype)
            assert rc == eik.EIK_OK, eik.last_error()
            ref, _ = gpu_util.solve_dev(eik, w, dtype=dtype)
            tol = 1e-12 if dtype == "f64" else 2.0 ** -20
            assert gpu_util.max_rel(got, ref) <= tol
    for w, s in ((W.smooth_sine(257), 16), (W.config(1), 8)):  # FMSM: the same order, bit for bit
        rc, got, _ = noalloc(eik, w, method="fmsm", cell=s)
        assert rc == eik.EIK_OK, eik.last_error()
        ref, _ = gpu_util.solve_dev(eik, w, method="fmsm", cell=s)
        assert np.array_equal(got, ref)


def test_limits_are_refused(eik):
    import torch
    w = W.smooth_sine(33)
    u = np.full((33, 33), 7.0)
    o = eik._opts(eik.F64, "exact", 0, 0.0, False, None, False, 0, 0)  # host pointers
    F = np.ascontiguousarray(w["F"])
    src = np.ascontiguousarray(w["src"])
    rc = eik.lib.eik_solve_noalloc(33, 33, w["h"], F.ctypes.data, None, 1, src.ctypes.data, None,
                                   u.ctypes.data, ctypes.byref(o), None)
    assert rc == eik.EIK_EINVAL and (u == 7.0).all()
    # a grid whose h/F alone exceeds the scratch: refused before any device work
    n = 4097
    dev = torch.device("cuda:0")
    Fd = torch.ones((n, n), dtype=torch.float64, device=dev)
    ud = torch.full_like(Fd, 7.0)
    sd = torch.zeros(1, dtype=torch.int64, device=dev)
    o = eik._opts(eik.F64, "exact", 0, 0.0, True, eik._stream_of(True), False, 0, 0)
    rc = eik.lib.eik_solve_noalloc(n, n, 1.0 / (n - 1), Fd.data_ptr(), None, 1, sd.data_ptr(), None,
                                   ud.data_ptr(), ctypes.byref(o), None)
    assert rc == eik.EIK_EINVAL and b"scratch" in eik.lib.eik_last_error()
    assert bool((ud == 7.0).all())
