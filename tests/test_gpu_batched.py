"""GPU parity of batched solves (many problems of different sizes in one
persistent launch) against the CPU oracle, FP64 and FP32."""
import numpy as np
import pytest

import oracle as O
from paper_1110_6220_amd import workloads as W
from gpu_util import f32_bound, max_abs, max_rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eik():
    import torch
    assert torch.cuda.is_available()
    from paper_1110_6220_amd import eik as E
    return E


def batch_dev(ws, dtype):
    out = []
    for w in ws:
        d = to_dev(w, dtype)
        out.append(d)
    return out


def run_batched(eik, ws, **kw):
    print(f"[gpu] batched {len(ws)} problems {kw}", flush=True)
    dtype = kw.get("dtype", "f64")
    us, st = eik.eik_solve_batched(batch_dev(ws, dtype), **kw)
    return [u.double().cpu().numpy() for u in us], st


def test_small_batch_fp64_device_and_host(eik):
    ws = W.batch_bumps(count=24, seed=40, n_lo=17, n_hi=200)
    ws += [W.random_small(np.random.default_rng(41 + k), nx, ny, q_spread=0.2)
           for k, (nx, ny) in enumerate([(1, 1), (1, 50), (70, 1), (65, 66), (130, 33)])]
    refs = [O.fmm(O.Problem.from_workload(w)) for w in ws]
    got, st = run_batched(eik, ws)
    for w, g, U in zip(ws, got, refs):
        assert max_rel(g, U) <= 1e-12, w["name"]
    assert len(st) == len(ws) and all(s["cells"] >= 1 for s in st)
    # host pointers: same results
    probs = [dict(F=w["F"], h=w["h"], src=w["src"], q=w["q"], mask=w.get("mask")) for w in ws]
    hu, _ = eik.eik_solve_batched(probs)
    for w, g, U in zip(ws, hu, refs):
        assert max_rel(g, U) <= 1e-12, w["name"]


def test_small_batch_fp32_with_residual_check(eik):
    ws = W.batch_bumps(count=16, seed=42, n_lo=33, n_hi=300)
    got, st = run_batched(eik, ws, dtype="f32", residual_check=True)
    for w, g in zip(ws, got):
        U = O.fmm(O.Problem.from_workload(w))
        assert max_abs(g, U) <= f32_bound(w, U), w["name"]
    assert 0.0 <= st[0]["max_residual"]


def test_batch_band_groups(eik):
    """Batches under the band schedule: each problem has its own group of
    bands (own cursor, width a multiple of its own s h).  Exact results under
    the tuned width and under explicit widths and windows (the Theorem of
    Section 3.2.1: any order converges to the discrete solution); FHCM in a
    batch within the accuracy of the serial oracle FHCM."""
    ws = W.batch_bumps(count=20, seed=44, n_lo=17, n_hi=260)
    ws += [W.random_small(np.random.default_rng(45), 90, 70, obst=0.1, nsrc=2, q_spread=0.2),
           W.random_small(np.random.default_rng(46), 1, 40)]
    refs = [O.fmm(O.Problem.from_workload(w)) for w in ws]
    for kw in ({}, dict(band=0.05, band_window=3), dict(band=1e-9), dict(band=1e9, band_window=63),
               dict(band_cells=2.0, band_window=1)):
        got, st = run_batched(eik, ws, schedule="bands", **kw)
        for w, g, U in zip(ws, got, refs):
            assert max_rel(g, U) <= 1e-12, (w["name"], kw)
        if "band" in kw:
            assert all(s["band_used"] == kw["band"] for s in st)
        else:
            # a multiple of each problem's own cell crossing s h
            ratio = [s["band_used"] / (s["cell_used"] * w["h"]) for s, w in zip(st, ws)]
            assert min(ratio) > 0 and max(ratio) <= min(ratio) * (1 + 1e-12), ratio
            if "band_cells" in kw:
                assert abs(ratio[0] - kw["band_cells"]) <= 1e-12
        assert st[0]["band_steps"] > 0
    fh = [W.smooth_sine(97), W.smooth_sine(129, amp=0.99), W.gaussian_bumps(150, np.random.default_rng(47))]
    got, st = run_batched(eik, fh, method="fhcm", cell=16)
    for w, g in zip(fh, got):
        p = O.Problem.from_workload(w)
        U = O.fmm(p)
        Vo, _ = O.fhcm(p, 16)
        assert (g >= U * (1 - 1e-14)).all(), w["name"]
        assert np.abs(g - U).max() <= 10 * np.abs(Vo - U).max() + 1e-12, w["name"]


def test_few_workers(eik):
    """Fewer persistent waves than the FIFO has rings: the queue uses no
    more rings than there are waves to wait on them (every ring is served),
    for batches and single problems, under every schedule."""
    ws = W.batch_bumps(count=6, seed=48, n_lo=40, n_hi=150)
    refs = [O.fmm(O.Problem.from_workload(w)) for w in ws]
    for workers in (1, 2, 3, 5):
        for sched in ("coarse", "fifo", "bands"):
            got, _ = run_batched(eik, ws, workers=workers, schedule=sched, cell=16, timeout_ms=5000)
            for w, g, U in zip(ws, got, refs):
                assert max_rel(g, U) <= 1e-12, (workers, sched, w["name"])
    d = to_dev(ws[0])
    u, _ = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, workers=3, cell=16, timeout_ms=5000)
    assert max_rel(u.cpu().numpy(), refs[0]) <= 1e-12


def test_fmsm_batched_bitwise(eik):
    ws = W.batch_bumps(count=8, seed=43, n_lo=40, n_hi=180)
    got, _ = run_batched(eik, ws, method="fmsm", cell=16)
    for w, g in zip(ws, got):
        V, _ = O.fmsm(O.Problem.from_workload(w), 16)
        assert np.array_equal(g, V), w["name"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_256_instance_batch_sampled(eik, dtype):
    """The 256-instance Gaussian-bump batch (sides 65..1025) in one launch:
    sampled instances (the largest, the smallest and six more) against the
    oracle; every instance's FP64 fixed-point residual via the library's
    residual pass."""
    ws = W.config(4)
    got, st = run_batched(eik, ws, dtype=dtype, residual_check=True)
    sizes = np.array([w["nx"] for w in ws])
    pick = {int(sizes.argmax()), int(sizes.argmin())} | set(range(0, 256, 37))
    for k in sorted(pick):
        w = ws[k]
        U = O.fmm(O.Problem.from_workload(w))
        if dtype == "f64":
            assert max_rel(got[k], U) <= 1e-12, w["name"]
        else:
            assert max_abs(got[k], U) <= f32_bound(w, U), w["name"]
    if dtype == "f64":
        assert st[0]["max_residual"] <= 1e-13
    for w, g in zip(ws, got):
        assert np.isfinite(g).all()  # no obstacles: every node reachable
        assert (g[np.unravel_index(w["src"], g.shape)] == 0.0).all()


def test_batch_object_repeated_solves(eik):
    """eik.Batch marshals once; repeated solves (graph replay from the second
    on) give the oracle's results every time."""
    ws = W.batch_bumps(count=10, seed=44, n_lo=50, n_hi=260)
    refs = [O.fmm(O.Problem.from_workload(w)) for w in ws]
    b = eik.Batch([to_dev(w) for w in ws], graph=True)
    print("[gpu] Batch object, three solves", flush=True)
    for rep in range(3):
        for u in b.outputs:
            u.fill_(-1.0)
        st = b.solve()
        assert st[0]["graph_replayed"] == (1 if rep else 0)
        for w, u, U in zip(ws, b.outputs, refs):
            assert max_rel(u.double().cpu().numpy(), U) <= 1e-12, (rep, w["name"])
