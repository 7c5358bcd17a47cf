"""Benchmark: solved grid nodes per second on one MI355X.

A step is one complete exact solve (every kernel of the path: validation and
initialisation, the coarse order, the persistent cell-sweeping kernel, the
statistics read-back) of the largest single-GPU workload: the 4097 x 4097
checkerboard of 16 x 16 squares with F ~ U[0.5, 2] per square and seeded
rectangular obstacles over >= 20% of the nodes, exit node at the corner
(0, 0), in FP64, with all inputs resident in device memory.  Only results
that pass the accuracy gate (max relative error <= 1e-12 against the CPU
oracle's Fast Marching solution, identical infinite sets) count.  Prints one
JSON line.

Beside the headline line's own fields (roofline of the solver kernel: its
algorithmic bytes over its device time against the HBM peak; span: the hop
depth D of the problem times the measured latency of one dependent sweep
step, against the same device time; LDS and VALU counters when the committed
profile matches the kernel source) it reports, from the same run:
  large_f32  the headline workload in FP32 with the FP64 residual recheck:
             max and L1 error against the FP64 oracle and the stated bound;
  smooth_1025
             the 1025 x 1025 smooth-speed workload F = 1 + 0.5 sin(2 pi x)
             sin(2 pi y), centre exit node, FP64 (roofline and span as above);
  batched  the 256-instance Gaussian-bump batch (sides 65..1025) solved in one
           persistent launch, against the same instances solved one launch each
           (batched_f32: the same in FP32, with max and L1 errors);
  serving  Kruskal-maze requests (sides 129..2049, FP32 with the FP64 residual
           recheck) through the continuous-batching server;
  early_termination, three_d, cells, fhcm_accuracy (see each function).

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
# LDS: 256 compute units x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4
BYTES_PER_NODE = {"f64": 17, "f32": 9}  # read F, read mask, write u
PROFILES = os.path.join(ROOT, "profiles")


def engine_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_1110_6220_amd", "csrc", "engine.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def counter_record(profile):
    """The COUNTERS record of a committed rocprofv3 counter summary (HBM bytes
    per launch from FETCH_SIZE / WRITE_SIZE scaled by a copy of known size;
    LDS bytes and instruction counts), or None when the summary is missing or
    was taken on another version of the kernel source."""
    path = os.path.join(PROFILES, profile)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("COUNTERS "):
            rec = json.loads(line[len("COUNTERS "):])
            if rec.get("engine_sha256_16") == engine_sha():
                return rec
    return None


def hop_depth(w):
    """Longest breadth-first hop count from the exit set over accessible
    nodes: the length D of the longest chain of dependent updates (a
    frontier-by-frontier search over the 4-neighbour grid)."""
    import numpy as np
    ny, nx = w["ny"], w["nx"]
    acc = np.ones(nx * ny, bool) if w.get("mask") is None else w["mask"].ravel().astype(bool)
    seen = ~acc
    # one guard column and row of "seen" nodes: neighbours never wrap
    seen = np.pad(seen.reshape(ny, nx), 1, constant_values=True).ravel()
    stride = nx + 2
    front = np.unique(np.asarray(w["src"], dtype=np.int64))
    front = (front // nx + 1) * stride + front % nx + 1
    seen[front] = True
    depth = 0
    while True:
        nb = np.concatenate([front - 1, front + 1, front - stride, front + stride])
        nb = nb[~seen[nb]]
        if nb.size == 0:
            return depth
        seen[nb] = True
        front = np.unique(nb)
        depth += 1


def roofline(n_nodes, dtype, kernel_s, profile=None):
    """HBM roofline of one solver launch: algorithmic bytes (read F, read the
    mask, write u once per node) over the kernel's device time, against the
    HBM peak; measured traffic and LDS figures from the committed counters."""
    bytes_alg = BYTES_PER_NODE[dtype] * n_nodes
    achieved = bytes_alg / kernel_s / 1e9
    rec = counter_record(profile) if profile else None
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": rec["traffic_bytes"] if rec and "traffic_bytes" in rec else None,
           "kernel": "k_solve", "kernel_us": kernel_s * 1e6, "bytes_per_launch": bytes_alg}
    if rec and "lds_bytes" in rec:
        lds = rec["lds_bytes"] / kernel_s / 1e9
        out["lds"] = {"bytes_per_launch": rec["lds_bytes"], "achieved_GBps": lds,
                      "peak_GBps": LDS_PEAK_GBS, "frac": lds / LDS_PEAK_GBS,
                      "bank_conflict_cycles_per_access": rec.get("bank_conflict_per_access"),
                      "valu_insts": rec.get("valu_insts"), "lds_insts": rec.get("lds_insts")}
    return out


def span(w, dtype, cell, kernel_s, D=None):
    """Span bound: the hop depth D of the problem times t_dep, the measured
    latency of one dependent anti-diagonal step of the cell sweep (one wave
    alone), against the solver kernel's device time."""
    from paper_1110_6220_amd import eik
    D = hop_depth(w) if D is None else D
    t_dep = eik.probe_step_latency(dtype, 64 if cell > 32 else 32, 400)
    return {"hop_depth": D, "t_dep_ns": t_dep * 1e9, "span_us": D * t_dep * 1e6,
            "kernel_us": kernel_s * 1e6, "frac": D * t_dep / kernel_s}


def f32_errors(got, U, h, D):
    """FP32 result against the FP64 oracle: max absolute and relative error,
    L1 error h^2 sum |u32 - U| over reachable nodes, and the stated bound
    (D + 2) 2^-24 max U (reading C20; D = hop depth)."""
    import numpy as np
    fin = np.isfinite(U)
    same = bool(np.array_equal(np.isfinite(got), fin))
    err = np.abs(got[fin].astype(np.float64) - U[fin])
    bound = (D + 2) * 2.0 ** -24 * float(U[fin].max())
    return {"max_abs": float(err.max()), "max_rel": float((err / np.maximum(U[fin], 1e-300)).max()),
            "L1": float(err.sum() * h * h), "bound": bound, "hop_depth": D,
            "share_of_bound": float(err.max()) / bound, "same_infinite_set": same,
            "passed": same and float(err.max()) <= bound}


def timed_solves(w, dtype, steps, warmup, graph=True, cell=0, residual_check=False):
    """`steps` complete solves of workload w after `warmup` untimed ones, with
    inputs resident on the device; returns (seconds, per-step kernel seconds,
    last stats, the result as float64)."""
    import torch

    from paper_1110_6220_amd import eik
    d = _to_dev(w, dtype)
    u = torch.empty_like(d["F"])
    torch.cuda.synchronize()

    def step():
        return eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"), u_out=u, dtype=dtype,
                             cell=cell, graph=graph, residual_check=residual_check)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kernel_s, stats = [], None
    t0 = time.perf_counter()
    for _ in range(steps):
        _, stats = step()
        kernel_s.append(stats["kernel_seconds"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, kernel_s, stats, u.double().cpu().numpy()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cell", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU oracle baseline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sub-records (batched, serving, studies)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-comparator", action="store_true",
                    help="batched: skip the one-launch-per-instance comparator (profiling runs)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step's kernels one by one instead of replaying the "
                         "captured HIP graph of the solve")
    ap.add_argument("--only", choices=["smooth_1025", "large_f32", "batched", "batched_f32", "serving",
                                       "early_termination", "three_d", "cells", "fhcm_accuracy"],
                    help="run one of the sub-records alone and print its JSON (no headline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on a single device)", file=sys.stderr)
        sys.exit(2)
    graph = not args.no_graph
    if args.only:
        runs = {"smooth_1025": lambda: bench_smooth(args.steps, args.warmup, graph),
                "large_f32": lambda: bench_large_f32(args.warmup, graph),
                "batched": lambda: bench_batched("f64", graph=graph, comparator=not args.no_comparator),
                "batched_f32": lambda: bench_batched("f32", graph=graph,
                                                     comparator=not args.no_comparator),
                "serving": lambda: bench_serving(args.serve_requests),
                "early_termination": bench_early_termination, "three_d": bench_3d,
                "cells": bench_cells, "fhcm_accuracy": bench_fhcm_accuracy}
        print(json.dumps({args.only: runs[args.only]()}), flush=True)
        return

    import numpy as np
    import torch

    import oracle
    from paper_1110_6220_amd import workloads

    # headline: the 4097^2 checkerboard with obstacles, FP64, exact method
    w = workloads.config(3)
    n_nodes = w["nx"] * w["ny"]
    elapsed, kernel_s, stats, got = timed_solves(w, "f64", args.steps, args.warmup, graph, args.cell)
    ms_per_step = 1e3 * elapsed / args.steps
    print(f"[bench] headline: {ms_per_step:.2f} ms per step", file=sys.stderr, flush=True)

    if args.copy_probe:
        # a plain copy of known size, for scaling the HBM byte counters
        dev = torch.device("cuda:0")
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev)  # 512 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # accuracy gate against the CPU oracle (Fast Marching, FP64)
    t_cpu0 = time.perf_counter()
    U = oracle.fmm(oracle.Problem.from_workload(w))
    t_fmm = time.perf_counter() - t_cpu0
    fin = np.isfinite(U)
    same_inf = bool(np.array_equal(np.isfinite(got), fin))
    rel = float((np.abs(got[fin] - U[fin]) / np.maximum(U[fin], 1e-300)).max())
    passed = same_inf and rel <= 1e-12

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
    D = hop_depth(w)
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "4097x4097 checkerboard of 16x16 squares, F ~ U[0.5, 2] per square (seed 3), "
                        "rectangular obstacles over >= 20% of the nodes (seed 33), exit node at the "
                        "corner (0, 0), exact method",
            "nx": w["nx"], "ny": w["ny"], "cell": int(stats["cell_used"]),
            "cells": int(stats["cells"]), "schedule": "coarse",
            "obstacle_share": float(1.0 - w["mask"].mean()),
            "launch": "HIP graph replay" if stats["graph_replayed"] else "stream",
            "parallelism": "single GPU",
        },
        "accuracy": {"max_rel_err_vs_fmm": rel, "tolerance": 1e-12, "same_infinite_set": same_inf,
                     "passed": passed},
        "roofline": roofline(n_nodes, "f64", avg_kernel, "k_solve_checker4097_f64.md"),
        "span": span(w, "f64", int(stats["cell_used"]), avg_kernel, D),
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
            "sample": f"Fast Marching (binary heap) on the same 4097x4097 problem, {reps} runs, "
                      f"{t_sum:.1f} s",
        },
    }
    if not args.no_extras:
        studies = [("large_f32", lambda: bench_large_f32(args.warmup, graph, U=U, D=D)),
                   ("smooth_1025", lambda: bench_smooth(args.steps, args.warmup, graph)),
                   ("batched", lambda: bench_batched("f64", graph=graph)),
                   ("batched_f32", lambda: bench_batched("f32", graph=graph)),
                   ("serving", lambda: serving_in_own_process(args.serve_requests)),
                   ("early_termination", bench_early_termination), ("three_d", bench_3d),
                   ("cells", bench_cells), ("fhcm_accuracy", bench_fhcm_accuracy)]
        for name, fn in studies:
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            line[name] = fn()
    print(json.dumps(line), flush=True)


def serving_in_own_process(count):
    """The serving record in a process of its own, as a server would run:
    a process that has replayed HIP graphs before it creates the server
    serves with a p99 about twice as high (measured; most likely two lanes
    then share one of the runtime's four hardware queues, where one lane's
    persistent launch holds up the other's work)."""
    import subprocess
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--only", "serving",
           "--serve-requests", str(count)]
    r = subprocess.run(cmd, cwd=ROOT, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"serving record failed (exit {r.returncode})")
    rec = json.loads(r.stdout.strip().splitlines()[-1])["serving"]
    rec["process"] = "own process (started by bench.py)"
    return rec


def bench_smooth(steps=20, warmup=3, graph=True):
    """The 1025 x 1025 smooth-speed workload F = 1 + 0.5 sin(2 pi x)
    sin(2 pi y) on [0, 1]^2 with the exit node at the centre, FP64, exact
    method: complete solves with device-resident inputs, gated at 1e-12
    against the oracle's Fast Marching; roofline and span of the solver
    kernel."""
    import numpy as np

    import oracle
    from paper_1110_6220_amd import workloads
    w = workloads.config(2)
    n = w["nx"] * w["ny"]
    elapsed, kernel_s, st, got = timed_solves(w, "f64", steps, warmup, graph)
    U = oracle.fmm(oracle.Problem.from_workload(w))
    rel = _max_rel(got, U)
    avg = float(np.mean(kernel_s))
    return {"workload": "1025x1025 smooth speed F=1+0.5 sin(2pi x) sin(2pi y) on [0,1]^2, "
                        "point source at the centre, exact method, FP64",
            "value": n * steps / elapsed if rel <= 1e-12 else 0.0, "unit": "nodes/s",
            "ms_per_step": 1e3 * elapsed / steps, "cell": int(st["cell_used"]),
            "max_rel_err_vs_fmm": rel, "AvHR": st["AvHR"], "AvS": st["AvS"],
            "roofline": roofline(n, "f64", avg, "k_solve_sine1025_f64.md"),
            "span": span(w, "f64", int(st["cell_used"]), avg)}


def bench_large_f32(warmup=3, graph=True, reps=5, U=None, D=None):
    """The headline workload in FP32 storage (FP64 two-sided branch) with the
    FP64 residual recheck: median wall time of `reps` solves, the max and L1
    error against the FP64 oracle and the stated bound (reading C20)."""
    import numpy as np

    import oracle
    from paper_1110_6220_amd import workloads
    w = workloads.config(3)
    n = w["nx"] * w["ny"]
    ts = []
    st, got = None, None
    for _ in range(reps):
        elapsed, kernel_s, st, got = timed_solves(w, "f32", 1, warmup if not ts else 0, graph,
                                                  residual_check=True)
        ts.append(elapsed)
    if U is None:
        U = oracle.fmm(oracle.Problem.from_workload(w))
    if D is None:
        D = hop_depth(w)
    err = f32_errors(got, U, w["h"], D)
    ok = err["passed"] and (st["fell_back_to_f64"] or 0.0 <= st["max_residual"] <= 4 * 2.0 ** -24)
    ms = float(np.median(ts)) * 1e3
    return {"workload": "the headline workload (4097x4097 checkerboard with obstacles) in FP32 with "
                        "the FP64 residual recheck",
            "value": n / ms * 1e3 if ok else 0.0, "unit": "nodes/s", "ms": ms,
            "kernel_ms": st["kernel_seconds"] * 1e3, "cell": int(st["cell_used"]),
            "max_residual": st["max_residual"], "fell_back_to_f64": int(st["fell_back_to_f64"]),
            "errors_vs_fp64_oracle": err,
            "roofline": roofline(n, "f32", st["kernel_seconds"])}


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


def bench_batched(dtype, reps=5, graph=True, comparator=True):
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

    def batch():  # statistics are read once after the timed solves
        plan.solve(stats=False)
        out["u"] = plan.outputs

    batch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        batch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / reps
    out["st"] = plan.stats()
    t_seq = float("nan")
    if comparator:  # the plain path: one launch sequence per instance
        t = time.perf_counter()
        for d in ds:
            eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, dtype=dtype)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t
    replayed = bool(out["st"][0]["graph_replayed"])
    # accuracy gate on sampled instances (largest, smallest, every 51st)
    sizes = np.array([w["nx"] for w in ws])
    pick = sorted({int(sizes.argmax()), int(sizes.argmin())} | set(range(0, 256, 51)))
    worst, passed, errs = 0.0, True, []
    for k in pick:
        U = oracle.fmm(oracle.Problem.from_workload(ws[k]))
        got = out["u"][k].double().cpu().numpy()
        if dtype == "f64":
            worst = max(worst, _max_rel(got, U))
            passed = passed and worst <= 1e-12
        else:  # FP32: max and L1 error against the FP64 oracle, bound of reading C20
            e = f32_errors(got, U, ws[k]["h"], hop_depth(ws[k]))
            errs.append({"instance": k, "side": ws[k]["nx"], **e})
            worst = max(worst, e["share_of_bound"])
            passed = passed and e["passed"]
    sts = out["st"]
    st = sts[0]
    cells = sum(x["cells"] for x in sts)
    acc = {"sampled": len(pick), "passed": passed}
    if dtype == "f64":
        acc["max_rel_err_vs_fmm_sampled"] = worst
    else:
        acc.update(worst_share_of_f32_bound=worst,
                   max_abs=max(e["max_abs"] for e in errs), max_L1=max(e["L1"] for e in errs),
                   per_instance=errs)
    return {
        "workload": "256 instances, sides ~U{65..1025}, F = clip(1 + 4 Gaussian bumps, 0.25, 2), "
                    "1-4 sources, one persistent launch",
        "nodes": n_nodes, "dtype": dtype,
        "value": n_nodes / t_batch if passed else 0.0, "unit": "nodes/s",
        "ms_per_batch": t_batch * 1e3,
        "launch": "HIP graph replay" if replayed else "stream",
        "one_launch_per_instance_ms": t_seq * 1e3,
        "speedup_vs_one_launch_per_instance": t_seq / t_batch,
        "kernel_ms": st["kernel_seconds"] * 1e3, "cell": int(st["cell_used"]),
        "AvHR": sum(x["cell_visits"] for x in sts) / cells,
        "AvS": sum(x["sweeps"] + x["checks"] for x in sts) / cells,
        "roofline": roofline(n_nodes, dtype, st["kernel_seconds"],
                             "k_solve_batch256_f64.md" if dtype == "f64" else None),
        "accuracy": acc,
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


def bench_serving(count, pool_size=128):
    """Maze requests through the continuous-batching server (FP32 with the
    FP64 residual recheck, host inputs, 64 GiB budget): saturated throughput
    (all `count` requests submitted at once), then Poisson arrivals at 0.25,
    0.5, 0.75 and 0.9 times the saturated request rate with p50/p99 latency
    (submission to completion, measured by the library), then all requests
    at once under a 256 MiB budget (admission waits for room).  The
    comparator is the plain path: the same requests solved one eik_solve
    call each, one after the other, at the same accuracy (FP32 with the
    residual recheck, host inputs).  Requests cycle through a pool of
    `pool_size` distinct seeded mazes (sides log-uniform in [129, 2049])."""
    import numpy as np

    import oracle
    from paper_1110_6220_amd import eik, workloads
    pool = workloads.maze_requests(min(count, pool_size), seed=5)
    for r in pool:  # the client holds its speeds in the server's precision
        r["F32"] = np.ascontiguousarray(r["F"], dtype=np.float32)
    reqs = [pool[k % len(pool)] for k in range(count)]
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

    # the plain path: one solve per request, host inputs, same accuracy
    for r in pool[:4]:
        eik.eik_solve(r["F32"], r["h"], r["src"], r["q"], r["mask"], dtype="f32", residual_check=True)
    solo = {}
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        t = time.perf_counter()
        eik.eik_solve(r["F32"], r["h"], r["src"], r["q"], r["mask"], dtype="f32", residual_check=True)
        solo.setdefault(id(r), time.perf_counter() - t)
    t_plain = time.perf_counter() - t0
    slowest_solo = max(solo.values())
    print(f"[bench] serving: plain path {count / t_plain:.0f} requests/s", file=sys.stderr, flush=True)

    points = []
    with eik.Server(64 << 30, dtype="f32", residual_check=True) as srv:
        for r in pool[:8]:  # warm-up: workspaces of every lane
            srv.wait(srv.submit(r["F32"], r["h"], r["src"], r["q"], r["mask"]))
        res, t_sat = submit_all(srv)
        rate = len(reqs) / t_sat
        allres = list(res)
        for frac in (0.25, 0.5, 0.75, 0.9):
            lam = frac * rate
            res2, t_poi = submit_all(srv, workloads.poisson_arrivals(len(reqs), lam, seed=5))
            allres += res2
            lat = np.array([st["seconds"] for _, st in res2])
            points.append({"load": frac, "rate_per_s": lam, "requests": len(reqs),
                           "value": nodes.sum() / t_poi,
                           "p50_ms": float(np.percentile(lat, 50) * 1e3),
                           "p99_ms": float(np.percentile(lat, 99) * 1e3),
                           "max_ms": float(lat.max() * 1e3)})
            print(f"[bench] serving: load {frac}: p50 {points[-1]['p50_ms']:.1f} ms, "
                  f"p99 {points[-1]['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
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
        e = f32_errors(res[k][0], U, reqs[k]["h"], hop_depth(reqs[k]))
        hops.append({"request": k, "side": reqs[k]["nx"], **e})
        checks.append(e["passed"])
    passed = certified and all(checks)
    half = points[1]
    return {
        "workload": f"{count} Kruskal-maze requests ({len(pool)} distinct), sides log-U[129, 2049], "
                    "corridors 4..16, FP32 + FP64 residual recheck, host inputs, 64 GiB budget",
        "nodes": float(nodes.sum()),
        "saturated_value": nodes.sum() / t_sat if passed else 0.0, "unit": "nodes/s",
        "saturated_requests_per_s": rate,
        "plain_path": {"requests_per_s": count / t_plain, "value": nodes.sum() / t_plain,
                       "slowest_request_alone_ms": slowest_solo * 1e3},
        "served_vs_plain": t_plain / t_sat,
        "poisson_rate_per_s": half["rate_per_s"],
        "poisson_value": half["value"] if passed else 0.0,
        "p50_ms": half["p50_ms"],
        "p99_ms": half["p99_ms"],
        "p99_at_0.25_vs_slowest_alone": points[0]["p99_ms"] / (slowest_solo * 1e3),
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
            rec = {}
            if dtype == "f64":
                ok = _max_rel(got, U) <= 1e-12
            else:
                rec = f32_errors(got, U, w["h"], 1024)  # hop depth of the centre source
                ok = rec["passed"]
            ms = statistics.median(ts) * 1e3
            out.append({"dtype": dtype, "cell": cell, "cell_used": int(st["cell_used"]), "ms": ms,
                        "nodes_per_s": n / ms * 1e3 if ok else 0.0, "AvHR": st["AvHR"], "AvS": st["AvS"],
                        "passed": ok, **({"errors_vs_fp64_oracle": rec} if rec else {})})
    return {"workload": "1025x1025 smooth speed F=1+0.5 sin(2pi x) sin(2pi y), centre exit node",
            "runs": out}


def bench_fhcm_accuracy():
    """FHCM's accuracy on the sinusoidal workloads of tables tab:sinu_1
    (a = 0.5, f = 10) and tab:sinu_2 (a = 0.99, f = 1), 1408^2, exit set at
    the centre: the error ratios of Section 4 -- calR = max E/e and rho =
    mean E/e over nodes with e != 0, R = max E / max e, where E = |V - u*| and
    e = |U - u*|, U the exact discrete solution and u* the exact solution on
    the 4x refined grid sampled at the nodes -- of the GPU FHCM under the
    serial heap order (the oracle's order, bit for bit) and under the
    concurrent band order, at 22 and 44 cells per side, beside the printed
    values (tests/golden/paper_tables_1408.txt) and the wall times."""
    import statistics

    import numpy as np
    import torch

    from paper_1110_6220_amd import eik, workloads
    printed = {}
    for ln in open(os.path.join(ROOT, "tests", "golden", "paper_tables_1408.txt")):
        f = ln.split()
        if len(f) == 6 and f[0] == "pt" and f[1].startswith("fhcm_"):
            printed[(float(f[2]), float(f[3]), int(f[4]), f[1][5:])] = float(f[5])

    def solve(w, **kw):
        d = _to_dev(w, "f64")
        u = torch.empty_like(d["F"])
        ts, st = [], None
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return u.cpu().numpy(), st, statistics.median(ts) * 1e3

    out = []
    for amp, freq in ((0.5, 10.0), (0.99, 1.0)):
        w = workloads.sinusoid_point(1408, amp, freq)
        truth = solve(workloads.sinusoid_point(4 * 1407 + 1, amp, freq))[0][::4, ::4]
        U, _, ms_exact = solve(w)
        e = np.abs(U - truth)
        pos = e != 0
        rec = {"workload": f"F = 1 + {amp} sin(2 pi {freq:g} x) sin(2 pi {freq:g} y), 1408^2, "
                           "centre exit set", "exact_ms": ms_exact, "runs": []}
        for cells in (22, 44):
            for sched in ("heap", "bands"):
                V, st, ms = solve(w, method="fhcm", cell=1408 // cells, schedule=sched)
                E = np.abs(V - truth)
                r = E[pos] / e[pos]
                rec["runs"].append({
                    "cells_per_side": cells, "schedule": sched, "ms": ms,
                    "calR": float(r.max()), "rho": float(r.mean()), "R": float(E.max() / e.max()),
                    "mon_pct": 100.0 * st["mon_ok"] / max(st["mon_checks"], 1),
                    "AvHR": st["AvHR"], "AvS": st["AvS"],
                    "printed": {k: printed.get((amp, freq, cells, k))
                                for k in ("rmax", "rho", "r", "mon")}})
        out.append(rec)
    return out


if __name__ == "__main__":
    main()
