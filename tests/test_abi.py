"""The C-ABI library loads and exports every entry point include/eik.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "eik.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(eik_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    assert "eik_solve" in names and "eik_solve_batched" in names and "eik_last_error" in names
    assert {"eik_serve_create", "eik_serve_submit", "eik_serve_poll", "eik_serve_wait",
            "eik_serve_cancel", "eik_serve_destroy"} <= set(names)


def test_library_exports_every_declared_symbol():
    from paper_1110_6220_amd import eik
    lib = ctypes.CDLL(eik.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(eik.EXPORTS)


def test_invalid_arguments_are_rejected_before_device_work():
    """Argument checks that need no device: sizes, spacing, enums, cell side."""
    import numpy as np
    from paper_1110_6220_amd import eik
    F = np.ones((4, 4))
    u = np.full((4, 4), 7.0)
    for kw in [dict(cell=3), dict(cell=65), dict(method="nope")]:
        try:
            eik.eik_solve(F, 0.1, [0], u_out=u, **kw)
        except (eik.EikError, KeyError):
            pass
        else:
            raise AssertionError(kw)
    for h in (0.0, -1.0, float("inf"), float("nan")):
        try:
            eik.eik_solve(F, h, [0], u_out=u)
        except eik.EikError as e:
            assert e.code == eik.EIK_EINVAL
        else:
            raise AssertionError(h)
    bad = F.copy()
    bad[1, 1] = 0.0
    for args in [(bad, 0.1, [0]), (F, 0.1, [16]), (F, 0.1, [-1])]:
        try:
            eik.eik_solve(*args, u_out=u)
        except eik.EikError as e:
            assert e.code == eik.EIK_EINVAL
        else:
            raise AssertionError(args)
    assert (u == 7.0).all()  # untouched


def test_sweep_arguments_are_rejected_before_device_work():
    """Whole-grid sweeping: option and input checks that need no device."""
    import numpy as np
    from paper_1110_6220_amd import eik
    F = np.ones((4, 4))
    u = np.full((4, 4), 7.0)
    bad = F.copy()
    bad[2, 3] = -1.0
    cases = [dict(F=F, src=[0], max_sweeps=-1), dict(F=F, src=[0], threshold=float("nan")),
             dict(F=bad, src=[0]), dict(F=F, src=[16]), dict(F=F, src=[])]
    for kw in cases:
        F_, src = kw.pop("F"), kw.pop("src")
        try:
            eik.eik_sweep(F_, 0.1, src, u_out=u, **kw)
        except eik.EikError as e:
            assert e.code == eik.EIK_EINVAL, kw
        else:
            raise AssertionError(kw)
    o = eik.SweepOpts(eik.F64, 2, 0, 0.0, 0, None)  # locking must be 0 or 1
    src = np.array([0], dtype=np.int64)
    st = eik.SweepStats()
    rc = eik.lib.eik_sweep_solve(4, 4, 0.1, F.ctypes.data, None, 1, src.ctypes.data, None,
                                 u.ctypes.data, o, None, None, st)
    assert rc == eik.EIK_EINVAL
    assert (u == 7.0).all()


def test_serving_arguments_are_checked_before_device_work():
    """Server entry points reject missing handles and invalid configurations
    without touching a device."""
    from paper_1110_6220_amd import eik
    L = eik.lib
    out = ctypes.c_void_p()
    assert L.eik_serve_create(None, ctypes.byref(out)) == eik.EIK_EINVAL
    for kw in [dict(cell=3), dict(lanes=17), dict(max_slots=-1)]:
        o = eik._opts(eik.F64, "exact", kw.get("cell", 0), 0.0, 0, None, 0, 0, 0)
        cfg = eik.ServeCfg(1 << 20, kw.get("max_slots", 0), kw.get("lanes", 0), o)
        assert L.eik_serve_create(ctypes.byref(cfg), ctypes.byref(out)) == eik.EIK_EINVAL, kw
        assert eik.last_error()
    t = ctypes.c_uint64()
    p = eik.Problem()
    st = eik.Stats()
    assert L.eik_serve_submit(None, ctypes.byref(p), ctypes.byref(t)) == eik.EIK_EINVAL
    assert L.eik_serve_poll(None, 1, ctypes.byref(st)) == eik.EIK_EINVAL
    assert L.eik_serve_wait(None, 1, ctypes.byref(st)) == eik.EIK_EINVAL
    assert L.eik_serve_cancel(None, 1) == eik.EIK_EINVAL
    assert L.eik_serve_destroy(None) == eik.EIK_EINVAL


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of eik_opts, eik_stats, eik_problem,
    eik_serve_cfg, eik_sweep_opts, eik_sweep_stats and eik3_stats have the sizes and
    field offsets the C header gives them (compiled with the host compiler;
    no device needed)."""
    import subprocess
    from paper_1110_6220_amd import eik
    structs = {"eik_opts": eik.Opts, "eik_stats": eik.Stats, "eik_problem": eik.Problem,
               "eik_serve_cfg": eik.ServeCfg, "eik_sweep_opts": eik.SweepOpts,
               "eik_sweep_stats": eik.SweepStats, "eik3_stats": eik.Stats3}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "eik.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_tuned_cell_table_covers_every_class():
    """Every (precision, batch, wall class) has a catch-all row, so the
    lookup always finds a cell side, and every side is a valid tile."""
    text = open(os.path.join(ROOT, "paper_1110_6220_amd", "csrc", "tuned_cells.h")).read()
    rows = re.findall(r"\{(\d), (\d), ([0-9 <]+), (\d), (\d+)\},", text)
    assert rows
    seen = set()
    for dt, batched, nmax, dense, cell in rows:
        assert int(cell) in (8, 16, 32, 64)
        if nmax.strip() == "1 << 30":
            seen.add((dt, batched, dense))
    assert seen == {(a, b, c) for a in "01" for b in "01" for c in "01"}


def test_negative_timeout_rejected():
    import numpy as np
    from paper_1110_6220_amd import eik
    u = np.full((4, 4), 7.0)
    try:
        eik.eik_solve(np.ones((4, 4)), 0.1, [0], u_out=u, timeout_ms=-1)
    except eik.EikError as e:
        assert e.code == eik.EIK_EINVAL
    else:
        raise AssertionError("negative timeout accepted")
    assert (u == 7.0).all()


def test_solve3_arguments_are_rejected_before_device_work():
    """3-D: shape, spacing, speed and source checks that need no device."""
    import numpy as np
    from paper_1110_6220_amd import eik
    F = np.ones((3, 4, 5))
    u = np.full(F.shape, 7.0)
    bad = F.copy()
    bad[1, 2, 3] = np.nan
    for method in ("exact", "fmsm"):
        for args in [(F, 0.0, [0]), (F, 0.1, [60]), (F, 0.1, [-1]), (bad, 0.1, [0]), (F, 0.1, [])]:
            try:
                eik.eik_solve3(args[0], args[1], args[2], u_out=u, method=method)
            except eik.EikError as e:
                assert e.code == eik.EIK_EINVAL, (method, args[1:])
            else:
                raise AssertionError((method, args[1:]))
    assert (u == 7.0).all()


def test_binding_rejects_mismatched_arrays():
    """The library takes plain pointers, so the binding checks array shapes,
    dtypes and layout against the grid before calling it (no device needed:
    host inputs are rejected before staging)."""
    import numpy as np
    import pytest
    from paper_1110_6220_amd import eik
    F2 = np.ones((6, 7))
    bad2 = [dict(u_out=np.empty((6, 6))), dict(u_out=np.empty((6, 7), dtype=np.float32)),
            dict(u_out=np.empty((7, 6)).T), dict(mask=np.ones((5, 7), dtype=np.uint8)),
            dict(q=[0.0, 0.1])]
    for kw in bad2:
        with pytest.raises(ValueError):
            eik.eik_solve(F2, 0.1, [3], **kw)
    F3 = np.ones((3, 4, 5))
    bad3 = [dict(u_out=np.empty((3, 4, 4))), dict(u_out=np.empty((3, 4, 5), dtype=np.float32)),
            dict(mask=np.ones((3, 4, 4), dtype=np.uint8)), dict(q=[0.0, 0.0, 0.0])]
    for kw in bad3:
        with pytest.raises(ValueError):
            eik.eik_solve3(F3, 0.1, [0, 7], **kw)
    ro = np.empty((6, 7))
    ro.setflags(write=False)
    with pytest.raises(ValueError):
        eik.eik_solve(F2, 0.1, [3], u_out=ro)
