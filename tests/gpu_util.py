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
