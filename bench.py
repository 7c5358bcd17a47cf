"""Benchmark: solved grid nodes per second on one MI355X.

A step is one complete exact solve (every kernel of the path: validation and
initialisation, the coarse Fast Marching order, the persistent cell-sweeping
kernel, the statistics read-back) of the 1025 x 1025 smooth-speed workload
F = 1 + 0.5 sin(2 pi x) sin(2 pi y) on [0, 1]^2 with a point source at the
centre, in FP64, with all inputs resident in device memory.  Only results that
pass the accuracy gate (max relative error <= 1e-12 against the CPU oracle's
Fast Marching solution) count.  Prints one JSON line.

Beside the headline line's own fields it reports, from the same run:
  batched  the 256-instance Gaussian-bump batch (sides 65..1025) solved in one
           persistent launch, against the same instances solved one launch each
           (batched_f32: the same in FP32);
  serving  Kruskal-maze requests (sides 129..2049, FP32 with the FP64 residual
           recheck) through the continuous-batching server under a 64 GiB
           budget: saturated throughput, then p50/p99 latency of Poisson
           arrivals at 0.25 / 0.5 / 0.75 / 0.9 of that request rate, then all
           at once under a 256 MiB budget (admission waits);
  early_termination
           the sweeping-method comparison of the Section 4 remark on stopping
           sweeping methods early, on this GPU: the 41 x 41 checkerboard at
           1312^2, FMSM with 41, 82 and 164 cells per side against whole-grid
           Fast Sweeping and Locking Sweeping stopped after the sweep count at
           which their error ratio R first reaches FMSM's (28 and 38 sweeps:
           table tab:check41_sweepMaxChange B, which the oracle reproduces in
           tests/test_oracle_sweeps.py), and run to convergence;
  three_d  the 3-D exact solver at 129^3 and 257^3 and 3-D FMSM at 129^3;
  cells    the headline workload at cell sides 8, 16, 32, 64 and the tuned
           one, FP64 and FP32;
  large    the 4097^2 checkerboard with rectangular obstacles, FP64 and FP32.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
BYTES_PER_NODE = {"f64": 17, "f32": 9}  # read F, read mask, write u
COUNTERS = os.path.join(ROOT, "profiles", "k_solve_sine1025_f64.md")


def measured_traffic(dtype):
    """HBM bytes per launch of the solver kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size), or None when it was taken on another version of the kernel."""
    import hashlib
    import json as _json
    if dtype != "f64" or not os.path.exists(COUNTERS):
        return None
    src = os.path.join(ROOT, "paper_1110_6220_amd", "csrc", "engine.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(COUNTERS):
        if line.startswith("COUNTERS "):
            rec = _json.loads(line[len("COUNTERS "):])
            if rec.get("engine_sha256_16") == sha:
                return rec["traffic_bytes"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cell", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU oracle baseline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and serving measurements")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step's kernels one by one instead of replaying the "
                         "captured HIP graph of the solve")
    ap.add_argument("--only", choices=["batched", "batched_f32", "serving", "early_termination", "three_d",
                                       "cells", "large"],
                    help="run one of the extra studies alone and print its JSON (no headline)")
    args = ap.parse_args()
    if args.only:
        runs = {"batched": lambda: bench_batched("f64", graph=not args.no_graph),
                "batched_f32": lambda: bench_batched("f32", graph=not args.no_graph),
                "serving": lambda: bench_serving(args.serve_requests),
                "early_termination": bench_early_termination, "three_d": bench_3d,
                "cells": bench_cells, "large": bench_large}
        print(json.dumps({args.only: runs[args.only]()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on a single device)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1110_6220_amd import eik, workloads

    w = workloads.config(2)
    n_nodes = w["nx"] * w["ny"]
    dev = torch.device("cuda:0")
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    F = torch.from_numpy(w["F"]).to(dev, tdt)
    src = torch.from_numpy(w["src"]).to(dev)
    q = torch.from_numpy(w["q"]).to(dev)
    u = torch.empty_like(F)
    torch.cuda.synchronize()

    graph = not args.no_graph

    def step():
        return eik.eik_solve(F, w["h"], src, q, None, u_out=u, dtype=args.dtype, cell=args.cell,
                             graph=graph)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernel_s = []
    stats = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, stats = step()
        kernel_s.append(stats["kernel_seconds"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    if args.copy_probe:
        # a plain copy of known size, for scaling the HBM byte counters
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev)  # 512 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # accuracy gate against the CPU oracle (Fast Marching, FP64)
    import oracle
    t_cpu0 = time.perf_counter()
    U = oracle.fmm(oracle.Problem.from_workload(w))
    t_fmm = time.perf_counter() - t_cpu0
    got = u.double().cpu().numpy()
    fin = np.isfinite(U)
    same_inf = bool(np.array_equal(np.isfinite(got), fin))
    rel = float((np.abs(got[fin] - U[fin]) / np.maximum(U[fin], 1e-300)).max())
    tol = 1e-12 if args.dtype == "f64" else (w["nx"] + w["ny"]) * 2.0 ** -24
    passed = same_inf and rel <= tol

    # CPU oracle baseline: Fast Marching on this workload, repeated within a
    # time budget on one host core (the method is serial)
    reps, t_sum = 1, t_fmm
    while t_sum < args.cpu_seconds:
        t1 = time.perf_counter()
        oracle.fmm(oracle.Problem.from_workload(w))
        t_sum += time.perf_counter() - t1
        reps += 1
    cpu_value = reps * n_nodes / t_sum

    avg_kernel = float(np.mean(kernel_s))
    bytes_alg = BYTES_PER_NODE[args.dtype] * n_nodes
    achieved = bytes_alg / avg_kernel / 1e9
    value = n_nodes * args.steps / elapsed if passed else 0.0
    line = {
        "metric": "solved grid nodes/s (err<=1e-12 vs FMM)",
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "1025x1025 smooth speed F=1+0.5 sin(2pi x) sin(2pi y) on [0,1]^2, "
                        "point source at the centre, exact method",
            "nx": w["nx"], "ny": w["ny"], "cell": int(stats["cell_used"]),
            "cells": int(stats["cells"]), "schedule": "coarse",
            "launch": "HIP graph replay" if stats["graph_replayed"] else "stream",
            "parallelism": "single GPU",
        },
        "accuracy": {"max_rel_err_vs_fmm": rel, "tolerance": tol, "passed": passed},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.dtype),
            "kernel": "k_solve",
            "kernel_us": avg_kernel * 1e6,
            "bytes_per_launch": bytes_alg,
        },
        "solver": {
            "AvHR": stats["AvHR"], "AvS": stats["AvS"],
            "cell_visits": int(stats["cell_visits"]), "sweeps": int(stats["sweeps"]),
            "checks": int(stats["checks"]),
        },
        "cpu_baseline": {
            "value": cpu_value,
            "unit": "nodes/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"Fast Marching (binary heap) on the same 1025x1025 problem, {reps} runs, "
                      f"{t_sum:.1f} s",
        },
    }
    if not args.no_extras:
        print("[bench] headline done; batched", file=sys.stderr, flush=True)
        line["batched"] = bench_batched("f64", graph=not args.no_graph)
        line["batched_f32"] = bench_batched("f32", graph=not args.no_graph)
        print("[bench] batched done; serving", file=sys.stderr, flush=True)
        line["serving"] = bench_serving(args.serve_requests)
        print("[bench] serving done; early termination", file=sys.stderr, flush=True)
        line["early_termination"] = bench_early_termination()
        print("[bench] early termination done; 3-D", file=sys.stderr, flush=True)
        line["three_d"] = bench_3d()
        print("[bench] 3-D done; cell sides", file=sys.stderr, flush=True)
        line["cells"] = bench_cells()
        print("[bench] cell sides done; 4097^2 checkerboard with obstacles", file=sys.stderr, flush=True)
        line["large"] = bench_large()
    print(json.dumps(line), flush=True)


def _to_dev(w, dtype):
    import torch
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    d = dict(F=torch.from_numpy(w["F"]).to(dev, tdt), h=w["h"],
             src=torch.from_numpy(w["src"]).to(dev), q=torch.from_numpy(w["q"]).to(dev))
    if w.get("mask") is not None:
        d["mask"] = torch.from_numpy(w["mask"]).to(dev)
    return d


def _max_rel(got, ref):
    import numpy as np
    fin = np.isfinite(ref)
    if not np.array_equal(np.isfinite(got), fin):
        return float("inf")
    return float((np.abs(got[fin] - ref[fin]) / np.maximum(ref[fin], 1e-300)).max()) if fin.any() else 0.0


def bench_batched(dtype, reps=5, graph=True):
    """256 instances in one launch vs one launch per instance (same kernels,
    same accuracy on sampled instances: FP64 <= 1e-12 relative to the
    oracle; FP32 within (nx + ny) 2^-24 max u, reported as the worst share of
    that bound), inputs resident on the device."""
    import numpy as np
    import torch

    import oracle
    from paper_1110_6220_amd import eik, workloads
    ws = workloads.config(4)
    n_nodes = sum(w["nx"] * w["ny"] for w in ws)
    ds = [_to_dev(w, dtype) for w in ws]
    for d in ds:  # fixed outputs: a repeated batch replays its captured graph
        d["u_out"] = torch.empty_like(d["F"])
    out = {}

    plan = eik.Batch(ds, dtype=dtype, graph=graph)  # marshalled once

    def batch():
        out["st"] = plan.solve()
        out["u"] = plan.outputs

    batch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        batch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for d in ds:
        eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, dtype=dtype)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    replayed = bool(out["st"][0]["graph_replayed"])
    # accuracy gate on sampled instances (largest, smallest, every 51st)
    sizes = np.array([w["nx"] for w in ws])
    pick = sorted({int(sizes.argmax()), int(sizes.argmin())} | set(range(0, 256, 51)))
    worst, passed = 0.0, True
    for k in pick:
        U = oracle.fmm(oracle.Problem.from_workload(ws[k]))
        got = out["u"][k].double().cpu().numpy()
        if dtype == "f64":
            worst = max(worst, _max_rel(got, U))
            passed = passed and worst <= 1e-12
        else:  # FP32: within (nx + ny) 2^-24 max u, identical infinite sets
            fin = np.isfinite(U)
            err = float(np.abs(got[fin] - U[fin]).max())
            bound = (ws[k]["nx"] + ws[k]["ny"]) * 2.0 ** -24 * float(U[fin].max())
            worst = max(worst, err / bound)
            passed = passed and err <= bound and bool(np.array_equal(np.isfinite(got), fin))
    st = out["st"][0]
    return {
        "workload": "256 instances, sides ~U{65..1025}, F = clip(1 + 4 Gaussian bumps, 0.25, 2), "
                    "1-4 sources, one persistent launch",
        "nodes": n_nodes, "dtype": dtype,
        "value": n_nodes / t_batch if passed else 0.0, "unit": "nodes/s",
        "ms_per_batch": t_batch * 1e3,
        "launch": "HIP graph replay" if replayed else "stream",
        "one_launch_per_instance_ms": t_seq * 1e3,
        "speedup_vs_one_launch_per_instance": t_seq / t_batch,
        "kernel_ms": st["kernel_seconds"] * 1e3, "AvHR": st["AvHR"], "AvS": st["AvS"],
        "accuracy": {("max_rel_err_vs_fmm_sampled" if dtype == "f64" else "worst_share_of_f32_bound"): worst,
                     "sampled": len(pick), "passed": passed},
    }


def bench_early_termination(reps=3):
    """Question 4 of the Section 4 remark on stopping sweeping methods early,
    on this GPU (FP64, inputs resident on the device, median wall time of
    `reps` calls, preparation included for every method)."""
    import statistics

    import torch

    from paper_1110_6220_amd import eik, workloads
    w = workloads.checkerboard_point(1312, 41)
    d = _to_dev(w, "f64")
    u = torch.empty_like(d["F"])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return statistics.median(ts) * 1e3, r

    out = {"workload": "41 x 41 checkerboard (F = 1 / 2), 1312 x 1312, exit set at the centre, FP64",
           "fmsm": [], "fsm": {}, "lsm": {}}
    # FMSM's R on this grid (table tab:checker_41) and the first Fast Sweeping
    # sweep whose R is at most that (table tab:check41_sweepMaxChange B)
    for cells, r_fmsm, k in ((41, 3.3991, 28), (82, 1.7662, 38), (164, 1.7123, 38)):
        ms, _ = timed(lambda: eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u,
                                            method="fmsm", cell=1312 // cells))
        out["fmsm"].append({"cells_per_side": cells, "cell": 1312 // cells, "ms": ms,
                            "R_fmsm": r_fmsm, "sweeps_to_same_R": k})
    for k in (28, 38, 0):
        for name, lock in (("fsm", False), ("lsm", True)):
            ms, r = timed(lambda: eik.eik_sweep(d["F"], d["h"], d["src"], d["q"], None, u_out=u,
                                                locking=lock, max_sweeps=k, threshold=-1.0 if k else 0.0))
            key = str(k) if k else f"converged ({r[3]['sweeps']} sweeps)"
            out[name][key] = {"ms": ms, "tiles_swept": r[3]["tiles_swept"],
                              "tiles_skipped": r[3]["tiles_skipped"]}
    ms, _ = timed(lambda: eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u))
    out["exact_ms"] = ms
    best = min(f["ms"] for f in out["fmsm"][1:])
    out["fmsm_82_vs_early_fsm_38"] = out["fsm"]["38"]["ms"] / out["fmsm"][1]["ms"]
    out["fmsm_82_vs_early_lsm_38"] = out["lsm"]["38"]["ms"] / out["fmsm"][1]["ms"]
    out["fmsm_best_of_82_164_ms"] = best
    return out


def bench_3d(sizes=(129, 257), reps=3):
    """The 3-D exact solver (eik_solve3) on smooth speeds
    F = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z) over the unit cube with a
    centre exit node: FP64, inputs resident on the device, median of `reps`
    calls; every result checked against the oracle's 3-D Fast Marching,
    whose single-core time is reported beside it.  At the first size also
    3-D FMSM (eik_fmsm3), checked bit for bit against the oracle's."""
    import statistics

    import numpy as np
    import torch

    import oracle
    from paper_1110_6220_amd import eik, workloads
    out = []
    for n in sizes:
        w = workloads.sine3(n, n, n, 0.5)
        dev = torch.device("cuda:0")
        F = torch.from_numpy(w["F"]).to(dev)
        src = torch.from_numpy(w["src"]).to(dev)
        q = torch.from_numpy(w["q"]).to(dev)
        u = torch.empty_like(F)
        eik.eik_solve3(F, w["h"], src, q, None, u_out=u)
        torch.cuda.synchronize()
        ts, st = [], None
        for _ in range(reps):
            t = time.perf_counter()
            _, st = eik.eik_solve3(F, w["h"], src, q, None, u_out=u)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        got = u.cpu().numpy()
        t = time.perf_counter()
        ref = oracle.fmm3(oracle.Problem3.from_workload(w))
        t_cpu = time.perf_counter() - t
        ms = statistics.median(ts) * 1e3
        out.append({"n": n, "nodes": n ** 3, "ms": ms, "nodes_per_s": n ** 3 / ms * 1e3,
                    "rounds_ms": st["rounds_seconds"] * 1e3, "rounds": st["rounds"],
                    "cells": st["cells"], "visits_per_cell": st["cell_visits"] / st["cells"],
                    "sweeps_per_visit": st["sweeps"] / max(st["cell_visits"], 1),
                    "max_rel_err_vs_fmm": _max_rel(got, ref),
                    # algorithmic bytes: read F, write u once (16 B/node)
                    "alg_GBps_over_rounds": 16.0 * n ** 3 / st["rounds_seconds"] / 1e9,
                    "cpu_oracle_fmm_nodes_per_s": n ** 3 / t_cpu})
        print(f"[bench] 3-D {n}^3: {ms:.2f} ms", file=sys.stderr, flush=True)
        if n == sizes[0]:
            # FMSM (cells of 8^3 nodes) on the same problem, checked bit for bit
            eik.eik_solve3(F, w["h"], src, q, None, u_out=u, method="fmsm")
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                _, sf = eik.eik_solve3(F, w["h"], src, q, None, u_out=u, method="fmsm")
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            V, so = oracle.fmsm3(oracle.Problem3.from_workload(w), 8)
            fin = np.isfinite(ref) & (ref > 0.0)  # relative to nonzero exact values
            out[-1]["fmsm"] = {"ms": statistics.median(ts) * 1e3, "levels": sf["rounds"],
                               "sweeps_per_cell": sf["sweeps"] / sf["cells"],
                               "bitwise_equal_oracle": bool(np.array_equal(u.cpu().numpy(), V)),
                               "max_rel_above_exact": float(((V[fin] - ref[fin]) / ref[fin]).max())}
            print(f"[bench] 3-D FMSM {n}^3: {out[-1]['fmsm']['ms']:.2f} ms", file=sys.stderr, flush=True)
    return out


def _hop_depth(w):
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    ny, nx = w["ny"], w["nx"]
    m = w["mask"].astype(bool)
    idx = np.arange(nx * ny).reshape(ny, nx)
    a = m[:, 1:] & m[:, :-1]
    b = m[1:, :] & m[:-1, :]
    r = np.concatenate([idx[:, 1:][a], idx[1:, :][b]])
    c = np.concatenate([idx[:, :-1][a], idx[:-1, :][b]])
    G = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(nx * ny, nx * ny)).tocsr()
    d = shortest_path(G, directed=False, unweighted=True, indices=int(w["src"][0]))
    return int(d[np.isfinite(d)].max())


def bench_serving(count):
    """Maze requests through the server: saturated throughput, then Poisson
    arrivals at 0.25, 0.5, 0.75 and 0.9 times the saturated request rate
    (latency = submission to completion, measured by the library); then the
    same requests at once through a 256 MiB budget, which makes admission
    wait for room."""
    import numpy as np

    import oracle
    from paper_1110_6220_amd import eik, workloads
    reqs = workloads.maze_requests(count, seed=5)
    for r in reqs:  # the client holds its speeds in the server's precision
        r["F32"] = np.ascontiguousarray(r["F"], dtype=np.float32)
    nodes = np.array([r["nx"] * r["ny"] for r in reqs], dtype=np.float64)

    def submit_all(srv, arrivals=None):
        tk = []
        t0 = time.perf_counter()
        for k, r in enumerate(reqs):
            if arrivals is not None:
                dt = arrivals[k] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            tk.append(srv.submit(r["F32"], r["h"], r["src"], r["q"], r["mask"]))
        res = [srv.wait(x) for x in tk]
        return res, time.perf_counter() - t0

    points = []
    with eik.Server(64 << 30, dtype="f32", residual_check=True) as srv:
        for r in reqs[:8]:  # warm-up: workspaces of every lane
            srv.wait(srv.submit(r["F32"], r["h"], r["src"], r["q"], r["mask"]))
        res, t_sat = submit_all(srv)
        rate = len(reqs) / t_sat
        allres = list(res)
        for frac in (0.25, 0.5, 0.75, 0.9):
            lam = frac * rate
            res2, t_poi = submit_all(srv, workloads.poisson_arrivals(len(reqs), lam, seed=5))
            allres += res2
            lat = np.array([st["seconds"] for _, st in res2])
            points.append({"load": frac, "rate_per_s": lam, "value": nodes.sum() / t_poi,
                           "p50_ms": float(np.percentile(lat, 50) * 1e3),
                           "p99_ms": float(np.percentile(lat, 99) * 1e3)})
    with eik.Server(256 << 20, dtype="f32", residual_check=True) as srv:
        res3, t_small = submit_all(srv)
        allres += res3
        lat3 = np.array([st["seconds"] for _, st in res3])
    # accuracy: every request certified by the FP64 residual recheck (or
    # re-solved in FP64); two requests against the oracle within the FP32 bound
    certified = all(st["fell_back_to_f64"] or 0.0 <= st["max_residual"] <= 4 * 2.0 ** -24
                    for _, st in allres)
    checks, hops = [], []
    for k in (0, int(np.argmax(nodes))):
        U = oracle.fmm(oracle.Problem.from_workload(reqs[k]))
        fin = np.isfinite(U)
        err = float(np.abs(res[k][0].astype(np.float64)[fin] - U[fin]).max())
        D = _hop_depth(reqs[k])
        hops.append({"request": k, "side": reqs[k]["nx"], "hop_depth": D})
        bound = (D + 2) * 2.0 ** -24 * float(U[fin].max())
        checks.append(err <= bound and np.array_equal(np.isfinite(res[k][0]), fin))
    passed = certified and all(checks)
    half = points[1]
    return {
        "workload": f"{count} Kruskal-maze requests, sides log-U[129, 2049], corridors 4..16, "
                    "FP32 + FP64 residual recheck, 64 GiB budget",
        "nodes": float(nodes.sum()),
        "saturated_value": nodes.sum() / t_sat if passed else 0.0, "unit": "nodes/s",
        "saturated_requests_per_s": rate,
        "poisson_rate_per_s": half["rate_per_s"],
        "poisson_value": half["value"] if passed else 0.0,
        "p50_ms": half["p50_ms"],
        "p99_ms": half["p99_ms"],
        "load_points": points,
        "budget_256MiB": {"value": nodes.sum() / t_small if passed else 0.0,
                          "requests_per_s": len(reqs) / t_small,
                          "p50_ms": float(np.percentile(lat3, 50) * 1e3),
                          "p99_ms": float(np.percentile(lat3, 99) * 1e3)},
        "checked_requests": hops,
        "fell_back_to_f64": int(sum(st["fell_back_to_f64"] for _, st in allres)),
        "accuracy": {"residual_certified": certified, "oracle_checks_passed": all(checks)},
    }


def bench_cells(reps=5):
    """The headline workload (1025^2 smooth speed, exit node at the centre) at
    every cell side 8, 16, 32, 64 and the tuned one (cell = 0), FP64 and FP32:
    median wall time of `reps` solves with device-resident inputs; FP64 gated
    at 1e-12 relative against the oracle's Fast Marching, FP32 within
    (nx + ny) 2^-24 max u."""
    import statistics

    import numpy as np
    import torch

    import oracle
    from paper_1110_6220_amd import eik, workloads
    w = workloads.config(2)
    U = oracle.fmm(oracle.Problem.from_workload(w))
    fin = np.isfinite(U)
    n = w["nx"] * w["ny"]
    out = []
    for dtype in ("f64", "f32"):
        d = _to_dev(w, dtype)
        u = torch.empty_like(d["F"])
        for cell in (8, 16, 32, 64, 0):
            def run():
                return eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u, dtype=dtype,
                                     cell=cell, graph=True)
            run()
            torch.cuda.synchronize()
            ts, st = [], None
            for _ in range(reps):
                t = time.perf_counter()
                _, st = run()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            got = u.double().cpu().numpy()
            if dtype == "f64":
                ok = _max_rel(got, U) <= 1e-12
            else:
                ok = bool(np.abs(got[fin] - U[fin]).max() <= (w["nx"] + w["ny"]) * 2.0 ** -24 * U[fin].max())
            ms = statistics.median(ts) * 1e3
            out.append({"dtype": dtype, "cell": cell, "cell_used": int(st["cell_used"]), "ms": ms,
                        "nodes_per_s": n / ms * 1e3 if ok else 0.0, "AvHR": st["AvHR"], "AvS": st["AvS"],
                        "passed": ok})
    return {"workload": "1025x1025 smooth speed F=1+0.5 sin(2pi x) sin(2pi y), centre exit node",
            "runs": out}


def bench_large(reps=3):
    """The 4097 x 4097 checkerboard (16 x 16 squares, F ~ U[0.5, 2] per square)
    with rectangular obstacles over >= 20% of the nodes, exit node at a corner,
    FP64 and FP32 (with the FP64 residual recheck): median wall time with
    device-resident inputs, gated against the oracle's Fast Marching (FP64:
    1e-12 relative; FP32: (nx + ny) 2^-24 max u)."""
    import statistics

    import numpy as np
    import torch

    import oracle
    from paper_1110_6220_amd import eik, workloads
    w = workloads.config(3)
    U = oracle.fmm(oracle.Problem.from_workload(w))
    fin = np.isfinite(U)
    n = w["nx"] * w["ny"]
    out = {"workload": "4097x4097 checkerboard of 16x16 squares with rectangular obstacles, "
                       "exit node at a corner",
           "obstacle_share": float(1.0 - w["mask"].mean()),
           "unreachable_accessible_nodes": int((~fin & (w["mask"] != 0)).sum()), "runs": []}
    for dtype in ("f64", "f32"):
        d = _to_dev(w, dtype)
        u = torch.empty_like(d["F"])
        def run():
            return eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d["mask"], u_out=u, dtype=dtype,
                                 residual_check=dtype == "f32")
        run()
        torch.cuda.synchronize()
        ts, st = [], None
        for _ in range(reps):
            t = time.perf_counter()
            _, st = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        got = u.double().cpu().numpy()
        same_inf = bool(np.array_equal(np.isfinite(got), fin))
        if dtype == "f64":
            ok = same_inf and _max_rel(got, U) <= 1e-12
        else:
            ok = same_inf and bool(np.abs(got[fin] - U[fin]).max()
                                   <= (w["nx"] + w["ny"]) * 2.0 ** -24 * U[fin].max())
        ms = statistics.median(ts) * 1e3
        out["runs"].append({"dtype": dtype, "ms": ms, "nodes_per_s": n / ms * 1e3 if ok else 0.0,
                            "cell_used": int(st["cell_used"]), "AvHR": st["AvHR"], "AvS": st["AvS"],
                            "passed": ok})
    return out

if __name__ == "__main__":
    main()
