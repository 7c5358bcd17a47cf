"""Serial CPU oracle for the two-scale Eikonal methods (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use this package; the GPU library never imports, links or runs
it.  The arithmetic lives in ``eik_oracle.c`` (plain C, fp64,
``-ffp-contract=off``); this module only marshals numpy arrays.

Functions follow Chacon & Vladimirsky, "Fast two-scale methods for Eikonal
equations": Fast Marching (Algorithm FMM), Fast Sweeping (Algorithms
FSM_order, FSM), Locking Sweeping (Section 2 remark on locking flags), value
iteration, the Heap-Cell Methods (Section 3.2, Algorithms generic_LC_cells and
FHCM, eq. cell_value) and the Fast Marching-Sweeping Method (Algorithm FMSM).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eik_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the same source (used to
# check that the pins reject deliberately broken variants).
_LIB_OVERRIDE = os.environ.get("EIK_ORACLE_LIB")
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off"]


def build(march_native: bool = False) -> str:
    """Compile eik_oracle.c into liboracle.so with gcc."""
    flags = list(CFLAGS) + (["-march=native"] if march_native else [])
    cmd = ["gcc", *flags, "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double),
        ("F", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("nsrc", ctypes.c_int32),
        ("src", ctypes.c_void_p), ("q", ctypes.c_void_p),
    ]


class _Problem3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double), ("F", ctypes.c_void_p), ("mask", ctypes.c_void_p),
        ("nsrc", ctypes.c_int32), ("src", ctypes.c_void_p), ("q", ctypes.c_void_p),
    ]


class CellStats(ctypes.Structure):
    _fields_ = [
        ("cells", ctypes.c_int64), ("removals", ctypes.c_int64), ("sweeps", ctypes.c_int64),
        ("mon_checks", ctypes.c_int64), ("mon_ok", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        d = {f: int(getattr(self, f)) for f, _ in self._fields_}
        d["AvHR"] = self.removals / max(self.cells, 1)
        d["AvS"] = self.sweeps / max(self.cells, 1)
        d["Mon%"] = 100.0 * self.mon_ok / self.mon_checks if self.mon_checks else float("nan")
        return d


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB)
                                  or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Problem)
        vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
        L.orc_update.restype = ctypes.c_double
        L.orc_update.argtypes = [ctypes.c_double] * 3
        L.orc_fmm.argtypes = [P, vp, vp, i64p]
        L.orc_fsm.argtypes = [P, vp, ctypes.POINTER(i32)]
        L.orc_lsm.argtypes = [P, vp, ctypes.POINTER(i32)]
        P3 = ctypes.POINTER(_Problem3)
        L.orc3_update.restype = ctypes.c_double
        L.orc3_update.argtypes = [ctypes.c_double] * 4
        L.orc3_fmm.argtypes = [P3, vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.orc3_fsm.argtypes = [P3, vp, ctypes.POINTER(i32)]
        L.orc3_jacobi.argtypes = [P3, vp, ctypes.POINTER(i32)]
        L.orc3_residual.restype = ctypes.c_double
        L.orc3_residual.argtypes = [P3, vp, vp]
        L.orc3_fmsm.argtypes = [P3, i32, vp, vp, vp, ctypes.POINTER(CellStats)]
        L.orc3_fmsm_orderings.restype = i32
        L.orc3_fmsm_orderings.argtypes = [i32, i32]
        L.orc_sweep_init.argtypes = [P, vp, vp]
        L.orc_fsm_sweep.argtypes = [P, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.orc_lsm_sweep.argtypes = [P, vp, vp, i32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
        L.orc_jacobi.argtypes = [P, vp, ctypes.POINTER(i32)]
        L.orc_residual.restype = ctypes.c_double
        L.orc_residual.argtypes = [P, vp, vp]
        L.orc_hcm.argtypes = [P, i32, i32, vp, ctypes.POINTER(CellStats)]
        L.orc_fmsm.argtypes = [P, i32, vp, vp, vp, ctypes.POINTER(CellStats)]
        L.orc_tiling.restype = i32
        L.orc_tiling.argtypes = [i32, i32, vp]
        L.orc_fmsm_dirs.restype = i32
        L.orc_fmsm_dirs.argtypes = [i32]
        _lib = L
    return _lib


class Problem:
    """A boundary-value problem |grad u| F = 1, u = q on the source nodes."""

    def __init__(self, F, h, src, q=None, mask=None):
        F = np.ascontiguousarray(F, dtype=np.float64)
        self.ny, self.nx = F.shape
        self.h = float(h)
        self.F = F
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
        self.q = None if q is None else np.ascontiguousarray(np.atleast_1d(q), dtype=np.float64)
        self._c = _Problem(
            self.nx, self.ny, self.h, self.F.ctypes.data,
            None if self.mask is None else self.mask.ctypes.data,
            len(self.src), self.src.ctypes.data,
            None if self.q is None else self.q.ctypes.data)

    @classmethod
    def from_workload(cls, w: dict) -> "Problem":
        return cls(w["F"], w["h"], w["src"], w.get("q"), w.get("mask"))

    @property
    def c(self):
        return ctypes.byref(self._c)


def _check(rc: int, name: str) -> None:
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def update(a: float, b: float, delta: float) -> float:
    return lib().orc_update(a, b, delta)


def fmm(p: Problem, want_order: bool = False):
    V = np.empty((p.ny, p.nx))
    order = np.empty(p.nx * p.ny, dtype=np.int64) if want_order else None
    na = ctypes.c_int64(0)
    _check(lib().orc_fmm(p.c, V.ctypes.data, None if order is None else order.ctypes.data,
                         ctypes.byref(na)), "orc_fmm")
    return (V, order[: na.value]) if want_order else V


def fsm(p: Problem):
    V = np.empty((p.ny, p.nx))
    n = ctypes.c_int32(0)
    _check(lib().orc_fsm(p.c, V.ctypes.data, ctypes.byref(n)), "orc_fsm")
    return V, n.value


def lsm(p: Problem):
    V = np.empty((p.ny, p.nx))
    n = ctypes.c_int32(0)
    _check(lib().orc_lsm(p.c, V.ctypes.data, ctypes.byref(n)), "orc_lsm")
    return V, n.value


class Problem3:
    """A 3-D boundary-value problem; F has shape (nz, ny, nx) (x fastest)."""

    def __init__(self, F, h, src, q=None, mask=None):
        F = np.ascontiguousarray(F, dtype=np.float64)
        self.nz, self.ny, self.nx = F.shape
        self.h = float(h)
        self.F = F
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
        self.q = None if q is None else np.ascontiguousarray(np.atleast_1d(q), dtype=np.float64)
        self._c = _Problem3(
            self.nx, self.ny, self.nz, self.h, self.F.ctypes.data,
            None if self.mask is None else self.mask.ctypes.data,
            len(self.src), self.src.ctypes.data,
            None if self.q is None else self.q.ctypes.data)

    @classmethod
    def from_workload(cls, w: dict) -> "Problem3":
        return cls(w["F"], w["h"], w["src"], w.get("q"), w.get("mask"))

    @property
    def c(self):
        return ctypes.byref(self._c)


def update3(a: float, b: float, c: float, delta: float) -> float:
    return lib().orc3_update(a, b, c, delta)


def fmm3(p: Problem3, want_order: bool = False):
    V = np.empty((p.nz, p.ny, p.nx))
    order = np.empty(p.nx * p.ny * p.nz, dtype=np.int64) if want_order else None
    na = ctypes.c_int64(0)
    _check(lib().orc3_fmm(p.c, V.ctypes.data, None if order is None else order.ctypes.data,
                          ctypes.byref(na)), "orc3_fmm")
    return (V, order[: na.value]) if want_order else V


def fsm3(p: Problem3):
    V = np.empty((p.nz, p.ny, p.nx))
    n = ctypes.c_int32(0)
    _check(lib().orc3_fsm(p.c, V.ctypes.data, ctypes.byref(n)), "orc3_fsm")
    return V, n.value


def fmsm3(p: Problem3, s: int):
    """3-D FMSM on cells of s^3 nodes; returns (V, stats with the coarse
    order, coarse values, AvS)."""
    V = np.empty((p.nz, p.ny, p.nx))
    K = [(n + s - 1) // s for n in (p.nx, p.ny, p.nz)]
    J = K[0] * K[1] * K[2]
    order = np.empty(J, dtype=np.int64)
    cu = np.empty(J)
    st = CellStats()
    _check(lib().orc3_fmsm(p.c, int(s), V.ctypes.data, order.ctypes.data, cu.ctypes.data,
                           ctypes.byref(st)), "orc3_fmsm")
    return V, {"order": order, "coarse_u": cu.reshape(K[2], K[1], K[0]), **st.as_dict()}


def fmsm3_orderings(faces: int, thin_axes: int = 0) -> int:
    return lib().orc3_fmsm_orderings(int(faces), int(thin_axes))


def jacobi3(p: Problem3):
    V = np.empty((p.nz, p.ny, p.nx))
    n = ctypes.c_int32(0)
    _check(lib().orc3_jacobi(p.c, V.ctypes.data, ctypes.byref(n)), "orc3_jacobi")
    return V, n.value


def residual3(p: Problem3, V):
    V = np.ascontiguousarray(V, dtype=np.float64)
    r = np.empty_like(V)
    m = lib().orc3_residual(p.c, V.ctypes.data, r.ctypes.data)
    if m < 0:
        raise ValueError("orc3_residual: invalid problem")
    return m, r


def sweep_init(p: Problem, locking: bool = False):
    """Start of the sweeping methods: V (q on exit nodes, +inf elsewhere)
    and, for Locking Sweeping, the unlocked flags."""
    V = np.empty((p.ny, p.nx))
    unl = np.zeros((p.ny, p.nx), dtype=np.uint8) if locking else None
    _check(lib().orc_sweep_init(p.c, V.ctypes.data, None if unl is None else unl.ctypes.data),
           "orc_sweep_init")
    return V, unl


def fsm_sweep(p: Problem, V, sweep: int):
    """Fast Sweeping's sweep number `sweep` over the whole grid, in place.
    Returns (largest decrease, number of nodes that decreased)."""
    assert V.dtype == np.float64 and V.flags.c_contiguous and V.shape == (p.ny, p.nx)
    mx, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().orc_fsm_sweep(p.c, V.ctypes.data, int(sweep), ctypes.byref(mx), ctypes.byref(cnt)),
           "orc_fsm_sweep")
    return mx.value, cnt.value


def lsm_sweep(p: Problem, V, unl, sweep: int):
    """Locking Sweeping's sweep number `sweep`, in place (V and unlocked
    flags).  Returns (largest decrease, number of nodes that decreased)."""
    assert V.dtype == np.float64 and V.flags.c_contiguous and V.shape == (p.ny, p.nx)
    assert unl.dtype == np.uint8 and unl.flags.c_contiguous and unl.shape == (p.ny, p.nx)
    mx, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().orc_lsm_sweep(p.c, V.ctypes.data, unl.ctypes.data, int(sweep), ctypes.byref(mx),
                               ctypes.byref(cnt)), "orc_lsm_sweep")
    return mx.value, cnt.value


def jacobi(p: Problem):
    V = np.empty((p.ny, p.nx))
    n = ctypes.c_int32(0)
    _check(lib().orc_jacobi(p.c, V.ctypes.data, ctypes.byref(n)), "orc_jacobi")
    return V, n.value


def residual(p: Problem, V):
    V = np.ascontiguousarray(V, dtype=np.float64)
    r = np.empty_like(V)
    m = lib().orc_residual(p.c, V.ctypes.data, r.ctypes.data)
    if m < 0:
        raise ValueError("orc_residual: invalid problem")
    return m, r


def hcm(p: Problem, s: int, fast: bool = False):
    V = np.empty((p.ny, p.nx))
    st = CellStats()
    _check(lib().orc_hcm(p.c, int(s), int(bool(fast)), V.ctypes.data, ctypes.byref(st)),
           "orc_hcm")
    return V, st.as_dict()


def fhcm(p: Problem, s: int):
    return hcm(p, s, fast=True)


def fmsm(p: Problem, s: int):
    V = np.empty((p.ny, p.nx))
    Kx, Ky = tiling(p.nx, s)[0], tiling(p.ny, s)[0]
    order = np.empty(Kx * Ky, dtype=np.int64)
    cu = np.empty(Kx * Ky)
    st = CellStats()
    _check(lib().orc_fmsm(p.c, int(s), V.ctypes.data, order.ctypes.data, cu.ctypes.data,
                          ctypes.byref(st)), "orc_fmsm")
    return V, {"order": order, "coarse_u": cu.reshape(Ky, Kx), **st.as_dict()}


def tiling(n: int, s: int):
    K = lib().orc_tiling(int(n), int(s), None)
    lo = np.empty(K + 1, dtype=np.int32)
    lib().orc_tiling(int(n), int(s), lo.ctypes.data)
    return K, lo


def fmsm_dirs(sides: int) -> int:
    return lib().orc_fmsm_dirs(int(sides))
