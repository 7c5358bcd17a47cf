"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import numpy as np


def to_dev(w, dtype="f64"):
    import torch
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    d = dict(F=torch.from_numpy(w["F"]).to(dev, tdt), h=w["h"],
             src=torch.from_numpy(w["src"]).to(dev), q=torch.from_numpy(w["q"]).to(dev))
    if w.get("mask") is not None:
        d["mask"] = torch.from_numpy(w["mask"]).to(dev)
    return d


def solve_dev(eik, w, **kw):
    """eik_solve through the C ABI on device copies of workload w; returns
    (u as a float64 numpy array, stats dict)."""
    d = to_dev(w, kw.get("dtype", "f64"))
    print(f"[gpu] solve {w['name']} {w['nx']}x{w['ny']} {kw}", flush=True)
    u, st = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"), **kw)
    return u.double().cpu().numpy(), st


def approx_cases():
    """(workload, cell side) pairs of the approximate-method parity tests:
    the constant-speed point source, smooth speeds, random problems with
    obstacles and several exit nodes, and the paper's 352..1408 sinusoids
    (four-node centre source, whole boundary as exit set) and 11 x 11 and
    41 x 41 checkerboards."""
    from paper_1110_6220_amd import workloads as W
    rng = np.random.default_rng(21)
    cases = [(W.config(1), 16), (W.config(1), 8), (W.smooth_sine(97), 8), (W.smooth_sine(257), 16),
             (W.smooth_sine(257, amp=0.99), 32)]
    for _ in range(4):
        nx, ny = (int(v) for v in rng.integers(20, 120, size=2))
        cases.append((W.random_small(rng, nx, ny, obst=0.1, nsrc=int(rng.integers(1, 4)),
                                     q_spread=0.2), int(rng.choice([4, 8, 16]))))
    cases += [(W.sinusoid_point(352, 0.5, 10.0), 16), (W.sinusoid_point(704, 0.5, 10.0), 32),
              (W.sinusoid_boundary(352, 0.5, 10.0), 16), (W.sinusoid_boundary(704, 0.99, 1.0), 32),
              (W.sinusoid_boundary(1408, 0.5, 10.0), 64),
              (W.checkerboard_point(352, 11), 16), (W.checkerboard_point(656, 41), 8),
              # 164^2 coarse cells
              (W.checkerboard_point(1312, 41), 8)]
    return cases


def max_rel(got, ref):
    """Max relative difference over finite reference nodes; the sets of
    infinite nodes must agree exactly."""
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), "reachable sets differ"
    assert np.array_equal(got[~fin], ref[~fin])
    if not fin.any():
        return 0.0
    r, g = ref[fin], got[fin]
    return float((np.abs(g - r) / np.maximum(np.abs(r), 1e-300)).max())


def max_abs(got, ref):
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), "reachable sets differ"
    return float(np.abs(got[fin] - ref[fin]).max()) if fin.any() else 0.0


def hop_depth(w):
    """Longest breadth-first hop count from the exit set over accessible
    nodes (the dependency depth D of the FP32 error bound)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    ny, nx = w["ny"], w["nx"]
    m = np.ones((ny, nx), bool) if w.get("mask") is None else w["mask"].astype(bool)
    idx = np.arange(nx * ny).reshape(ny, nx)
    a = m[:, 1:] & m[:, :-1]
    b = m[1:, :] & m[:-1, :]
    r = np.concatenate([idx[:, 1:][a], idx[1:, :][b]])
    c = np.concatenate([idx[:, :-1][a], idx[:-1, :][b]])
    G = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(nx * ny, nx * ny)).tocsr()
    d = shortest_path(G, directed=False, unweighted=True, indices=np.unique(w["src"]))
    d = np.atleast_2d(d).min(axis=0)
    fin = np.isfinite(d)
    return int(d[fin].max()) if fin.any() else 0


def f32_bound(w, U):
    """Worst-case FP32 error: every update and the speed and h/F conversions
    round with relative error <= 2^-24, and the update is monotone and
    non-expansive, so errors add along the dependency chain:
    |u32 - U| <= (D + 2) 2^-24 max U."""
    fin = np.isfinite(U)
    return (hop_depth(w) + 2) * 2.0 ** -24 * float(U[fin].max())
