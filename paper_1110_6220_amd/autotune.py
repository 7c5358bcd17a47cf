"""Autotuner for the cell side of the exact method and for the band width
of the band schedule.

The exact method's result does not depend on the cell side (the Theorem of
Section 3.2.1 of Chacon & Vladimirsky: label-correcting on cells converges to
the solution of the discrete system for any decomposition), so the side is a
pure speed knob.  This script times every candidate side on synthetic problems
of each class (precision, single problem or batch, grid size, open grid or
dense walls) on the current device and writes the table the library compiles
in (csrc/tuned_cells.h).

The band schedule takes cells from the lowest bands of their cell values; a
band's width (in cell crossings s h at unit speed) and the number of bands
above the lowest that may start (the window) set how far the concurrent
order strays from the heap order of Section 3.2.2.  For the exact method that
is again speed only.  For FHCM it also moves the error, so a width qualifies
only if the FHCM result stays as close to the exact discrete solution as the
serial heap order's: max error over the samples at most 1.1 times the heap
order's, in the worse of two runs, both measured in FP64 (for the FP32 rows
too: FP32 rounding would mask the order's effect).  --bands times the candidates and
writes csrc/tuned_bands.h.

    python -m paper_1110_6220_amd.autotune --out paper_1110_6220_amd/csrc/tuned_cells.h
    python -m paper_1110_6220_amd.autotune --bands --out paper_1110_6220_amd/csrc/tuned_bands.h

Rebuild the library afterwards (__graft_entry__.build()).
"""
from __future__ import annotations

import argparse
import statistics
import time

import numpy as np

from . import workloads as W

CANDIDATES = (8, 16, 32, 64)
DENSE_WALLS = 0.03
# size buckets (largest side) per wall class
OPEN_BUCKETS = (160, 512, 1 << 30)
DENSE_BUCKETS = (512, 1 << 30)


def _open_samples(nmax_prev, nmax, batched, rng):
    lo = max(nmax_prev + 1, 33)
    hi = min(nmax, 2049)
    if batched:
        sides = rng.integers(lo, hi + 1, size=24 if hi <= 512 else 12)
        return [W.gaussian_bumps(int(n), rng) for n in sides]
    sides = sorted({lo, (lo + hi) // 2, hi})
    return [W.smooth_sine(int(n), 0.5) for n in sides] + [W.gaussian_bumps(int(hi), rng)]


def _dense_samples(nmax_prev, nmax, batched, rng):
    lo = max(nmax_prev + 1, 129)
    hi = min(nmax, 2049)
    count = 16 if batched else 3
    out = []
    for _ in range(count):
        n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        out.append(W.kruskal_maze(n, rng))
    return out


def _time(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return statistics.median(ts)


def tune(dtypes=("f64", "f32"), log=print):
    import torch

    from . import eik
    dev = torch.device("cuda:0")
    rows, notes = [], []
    for dt_code, dtype in enumerate(("f64", "f32")):
        if dtype not in dtypes:
            continue
        tdt = torch.float64 if dtype == "f64" else torch.float32
        for dense, buckets in ((0, OPEN_BUCKETS), (1, DENSE_BUCKETS)):
            prev = 0
            for nmax in buckets:
                for batched in (0, 1):
                    rng = np.random.default_rng(1000 + 10 * nmax % 997 + batched + 2 * dense)
                    ws = (_dense_samples if dense else _open_samples)(prev, nmax, batched, rng)
                    ds = []
                    for w in ws:
                        d = dict(F=torch.from_numpy(w["F"]).to(dev, tdt), h=w["h"],
                                 src=torch.from_numpy(w["src"]).to(dev),
                                 q=torch.from_numpy(w["q"]).to(dev))
                        if w.get("mask") is not None:
                            d["mask"] = torch.from_numpy(w["mask"]).to(dev)
                        ds.append(d)
                    times = {}
                    for cell in CANDIDATES:
                        if batched:
                            t = _time(lambda: eik.eik_solve_batched(ds, dtype=dtype, cell=cell))
                        else:
                            t = _time(lambda: [eik.eik_solve(d["F"], d["h"], d["src"], d["q"],
                                                             d.get("mask"), dtype=dtype, cell=cell)
                                               for d in ds])
                        times[cell] = t
                    best = min(times, key=times.get)
                    if batched:
                        # a batch's widest cell sets every wave's LDS: take
                        # the smallest side within 3% of the fastest
                        best = min(c for c in CANDIDATES if times[c] <= 1.03 * times[best])
                    rows.append((dt_code, batched, nmax, dense, best))
                    sides = [w["nx"] for w in ws]
                    note = (f"{dtype} batched={batched} dense={dense} n<={nmax if nmax < 1 << 30 else 'any'}"
                            f" ({len(ws)} problems, sides {min(sides)}..{max(sides)}): "
                            + ", ".join(f"{c}: {times[c] * 1e3:.2f} ms" for c in CANDIDATES)
                            + f" -> {best}")
                    notes.append(note)
                    log(note)
                prev = nmax
    return rows, notes


BAND_FACTORS = (0.5, 1.0, 2.0, 4.0, 8.0)
BAND_WINDOWS = (0, 1, 3)
FHCM_ERR_SLACK = 1.1


def _band_samples(batched, rng):
    if batched:
        sides = rng.integers(65, 514, size=16)
        return [W.gaussian_bumps(int(n), rng) for n in sides]
    return [W.smooth_sine(513, 0.5), W.gaussian_bumps(385, rng),
            W.sinusoid_point(352, 0.5, 10.0), W.checkerboard_point(352, 11)]


def tune_bands(dtypes=("f64", "f32"), log=print):
    """Rows (method, dtype code, batched, width in cell crossings, window)
    and notes with the measurements."""
    import torch

    from . import eik
    dev = torch.device("cuda:0")
    rows, notes = [], []
    for method, mcode in (("exact", 0), ("fhcm", 2)):
        for dt_code, dtype in enumerate(("f64", "f32")):
            if dtype not in dtypes:
                continue
            tdt = torch.float64 if dtype == "f64" else torch.float32
            for batched in (0, 1):
                # the same samples for both precisions (FHCM's choice rests on
                # FP64 errors either way)
                rng = np.random.default_rng(2000 + 7 * mcode + batched)
                ws = _band_samples(batched, rng)
                ds = []
                for w in ws:
                    d = dict(F=torch.from_numpy(w["F"]).to(dev, tdt), h=w["h"],
                             src=torch.from_numpy(w["src"]).to(dev),
                             q=torch.from_numpy(w["q"]).to(dev))
                    if w.get("mask") is not None:
                        d["mask"] = torch.from_numpy(w["mask"]).to(dev)
                    ds.append(d)

                ds64 = [dict(d, F=d["F"].double()) for d in ds]

                def solve_all(prec=dtype, **kw):
                    dd = ds if prec == dtype else ds64
                    if batched:
                        us, _ = eik.eik_solve_batched(dd, dtype=prec, method=method,
                                                      schedule="bands", **kw)
                        return us
                    return [eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"),
                                          dtype=prec, method=method, schedule="bands", **kw)[0]
                            for d in dd]

                heap_err = None
                if method == "fhcm":
                    # errors are taken in FP64 for both precisions (FP32
                    # rounding would mask the order's effect): the exact
                    # discrete solutions and the serial heap order's error
                    # over the samples
                    ex = [eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"))[0] for d in ds64]

                    def err(us):
                        return max(float((u.double() - e).abs().nan_to_num(0.0).max())
                                   for u, e in zip(us, ex))
                    heap_err = err([eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d.get("mask"),
                                                  method="fhcm", schedule="heap")[0] for d in ds64])
                times, errs = {}, {}
                for f in BAND_FACTORS:
                    for win in BAND_WINDOWS:
                        # an explicit width: f cell crossings of each problem
                        kw = dict(band_cells=f, band_window=win)
                        times[(f, win)] = _time(lambda: solve_all(**kw))
                        if heap_err is not None:
                            # the concurrent order varies from run to run:
                            # the worse of two runs
                            errs[(f, win)] = max(err(solve_all("f64", **kw)),
                                                 err(solve_all("f64", **kw))) / max(heap_err, 1e-300)
                ok = [c for c in times if heap_err is None or errs[c] <= FHCM_ERR_SLACK]
                if not ok:
                    ok = [(1.0, 0)]
                best = min(ok, key=times.get)
                rows.append((mcode, dt_code, batched, best[0], best[1]))
                sides = [w["nx"] for w in ws]
                note = (f"{method} {dtype} batched={batched} ({len(ws)} problems, sides "
                        f"{min(sides)}..{max(sides)}): "
                        + ", ".join(f"{c[0]:g}/{c[1]}: {times[c] * 1e3:.2f} ms"
                                    + (f" err x{errs[c]:.2f}" if c in errs else "")
                                    for c in sorted(times))
                        + f" -> {best[0]:g}/{best[1]}")
                notes.append(note)
                log(note)
    return rows, notes


def write_bands_header(path, rows, notes, device_name):
    lines = [
        "// Band widths of the band schedule, written by paper_1110_6220_amd/autotune.py",
        "// (--bands) on " + device_name + ".  Row: method (0 exact, 2 FHCM), dtype",
        "// (0 f64, 1 f32), batched (problems per launch > 1), width in cell",
        "// crossings s h, window.  Measurements (median of 3; width/window: time,",
        f"// FHCM: max error / the heap order's, worse of 2 runs, must be <= {FHCM_ERR_SLACK}):",
    ]
    lines += ["//   " + n for n in notes]
    lines += ["#pragma once", "namespace eik {", "struct TunedBand {", "  int method, dtype, batched;",
              "  double factor;", "  int window;", "};", "constexpr TunedBand kTunedBands[] = {"]
    for r in rows:
        lines.append(f"    {{{r[0]}, {r[1]}, {r[2]}, {r[3]!r}, {r[4]}}},")
    lines += ["};", "}  // namespace eik", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def write_header(path, rows, notes, device_name):
    lines = [
        "// Cell sides chosen by paper_1110_6220_amd/autotune.py on " + device_name + ".",
        "// Exact method only: its result does not depend on the cell side, so the",
        "// table changes speed, never results.  Row: dtype (0 f64, 1 f32), batched",
        "// (problems per launch > 1), largest side of the bucket, dense walls (wall",
        "// density >= kDenseWalls), cell side.  Measurements (median of 3):",
    ]
    lines += ["//   " + n for n in notes]
    lines += ["#pragma once", "namespace eik {", f"constexpr double kDenseWalls = {DENSE_WALLS};",
              "struct TunedCell {", "  int dtype, batched, nmax, dense, cell;", "};",
              "constexpr TunedCell kTunedCells[] = {"]
    for r in rows:
        nmax = "1 << 30" if r[2] >= 1 << 30 else str(r[2])
        lines.append(f"    {{{r[0]}, {r[1]}, {nmax}, {r[3]}, {r[4]}}},")
    lines += ["};", "}  // namespace eik", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True, help="header to write")
    ap.add_argument("--dtype", action="append", choices=["f64", "f32"])
    ap.add_argument("--bands", action="store_true", help="tune the band schedule instead")
    args = ap.parse_args()
    import torch
    dts = tuple(args.dtype or ("f64", "f32"))
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.bands:
        rows, notes = tune_bands(dts, log=log)
        write_bands_header(args.out, rows, notes, torch.cuda.get_device_name(0))
    else:
        rows, notes = tune(dts, log=log)
        write_header(args.out, rows, notes, torch.cuda.get_device_name(0))
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
