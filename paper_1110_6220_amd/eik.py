"""Python binding of libeik (argument marshalling only).

Every entry point forwards to the C ABI of ``include/eik.h`` in ``libeik.so``;
all computation happens in the library's HIP kernels.  numpy arrays are passed
as host pointers (the library stages them); torch tensors on a ROCm device are
passed as device pointers and the work is ordered on torch's current stream.
There is no fallback: if the library is not built, importing fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeik.so")

EIK_OK, EIK_EINVAL, EIK_ENOMEM, EIK_EDEVICE, EIK_EBUDGET, EIK_ENOTCONV, EIK_EBUSY = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
METHODS = {"exact": 0, "hcm": 0, "fmsm": 1, "fhcm": 2}
SCHEDULES = {"auto": 0, "coarse": 1, "bands": 2, "fifo": 3, "heap": 4}

# Every function include/eik.h declares.
EXPORTS = ("eik_solve", "eik_solve_batched", "eik_serve_create", "eik_serve_submit",
           "eik_serve_poll", "eik_serve_wait", "eik_serve_cancel", "eik_serve_destroy",
           "eik_sweep_solve", "eik_solve3", "eik_fmsm3", "eik_solve_noalloc", "eik_probe_step_latency",
           "eik_last_error")


class EikError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libeik error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("method", ctypes.c_int), ("cell", ctypes.c_int32),
                ("band", ctypes.c_double), ("device_ptrs", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("max_cell_visits", ctypes.c_uint64),
                ("residual_check", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("band_window", ctypes.c_int32), ("eager_publish", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("timeout_ms", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("residual_tol", ctypes.c_double),
                ("band_cells", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("kernel_seconds", ctypes.c_double),
                ("cells", ctypes.c_uint64), ("cell_visits", ctypes.c_uint64),
                ("sweeps", ctypes.c_uint64), ("checks", ctypes.c_uint64),
                ("band_steps", ctypes.c_uint64), ("mon_checks", ctypes.c_uint64),
                ("mon_ok", ctypes.c_uint64), ("max_residual", ctypes.c_double),
                ("cell_used", ctypes.c_int32), ("band_used", ctypes.c_double),
                ("fell_back_to_f64", ctypes.c_int32), ("cells_total", ctypes.c_uint64),
                ("graph_replayed", ctypes.c_int32), ("residual_f32", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        cells = max(int(self.cells), 1)
        d["AvHR"] = self.cell_visits / cells
        d["AvS"] = (self.sweeps + self.checks) / cells
        return d


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double),
                ("F", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("nsrc", ctypes.c_int32),
                ("src", ctypes.c_void_p), ("q", ctypes.c_void_p), ("u_out", ctypes.c_void_p)]


class SweepOpts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("locking", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("threshold", ctypes.c_double), ("device_ptrs", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class SweepStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("seconds", ctypes.c_double), ("tiles_swept", ctypes.c_int64),
                ("tiles_skipped", ctypes.c_int64)]


class Stats3(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("rounds_seconds", ctypes.c_double),
                ("rounds", ctypes.c_int32), ("cells", ctypes.c_int64),
                ("cell_visits", ctypes.c_int64), ("sweeps", ctypes.c_int64)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("opts", Opts)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(paper_1110_6220_amd/build.py) first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.eik_solve.argtypes = [i32, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp,
                            ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
    L.eik_solve_batched.argtypes = [i32, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                    ctypes.POINTER(Stats)]
    L.eik_serve_create.argtypes = [ctypes.POINTER(ServeCfg), ctypes.POINTER(vp)]
    L.eik_serve_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_uint64)]
    L.eik_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Stats)]
    L.eik_serve_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Stats)]
    L.eik_serve_cancel.argtypes = [vp, ctypes.c_uint64]
    L.eik_serve_destroy.argtypes = [vp]
    L.eik_solve3.argtypes = [i32, i32, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp, i32, vp,
                             ctypes.POINTER(Stats3)]
    L.eik_fmsm3.argtypes = [i32, i32, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp, i32, vp,
                             ctypes.POINTER(Stats3)]
    L.eik_sweep_solve.argtypes = [i32, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp,
                                  ctypes.POINTER(SweepOpts), vp, vp, ctypes.POINTER(SweepStats)]
    L.eik_solve_noalloc.argtypes = [i32, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp,
                                    ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
    L.eik_probe_step_latency.argtypes = [i32, i32, i32, ctypes.POINTER(ctypes.c_double)]
    L.eik_last_error.restype = ctypes.c_char_p
    return L


lib = _load()


def last_error() -> str:
    return lib.eik_last_error().decode()


def _check(rc: int) -> None:
    if rc != EIK_OK:
        raise EikError(rc, last_error())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _opts(dtype, method, cell, band, device, stream, residual_check, workers, max_cell_visits,
          band_window=0, eager_publish=False, schedule="auto", timeout_ms=0, graph=False,
          residual_tol=0.0, band_cells=0.0):
    return Opts(dtype, METHODS[method], int(cell), float(band), int(device),
                stream, int(max_cell_visits), int(bool(residual_check)), int(workers),
                int(band_window), int(bool(eager_publish)), SCHEDULES[schedule], int(timeout_ms),
                int(bool(graph)), float(residual_tol), float(band_cells))


def _check_arrays(shape, mask, q, nsrc, u_out, out_dtype, device):
    """The library takes plain pointers and cannot see buffer sizes: the
    arrays must match the grid before any call.  Raises ValueError."""
    shape = tuple(shape)
    if mask is not None and tuple(mask.shape) != shape:
        raise ValueError(f"mask has shape {tuple(mask.shape)}, the grid {shape}")
    if q is not None and (q.numel() if _is_torch(q) else q.size) != nsrc:
        raise ValueError(f"q has {q.numel() if _is_torch(q) else q.size} values for {nsrc} sources")
    if u_out is None:
        return
    if tuple(u_out.shape) != shape:
        raise ValueError(f"u_out has shape {tuple(u_out.shape)}, the grid {shape}")
    if u_out.dtype != out_dtype:
        raise ValueError(f"u_out has dtype {u_out.dtype}, expected {out_dtype}")
    if device is not None:
        if not _is_torch(u_out) or u_out.device != device or not u_out.is_contiguous():
            raise ValueError("u_out must be a contiguous tensor on the inputs' device")
    elif _is_torch(u_out) or not u_out.flags.c_contiguous or not u_out.flags.writeable:
        raise ValueError("u_out must be a writeable C-contiguous numpy array for host inputs")


def _marshal(F, h, src, q, mask, u_out, dtype):
    """Returns (Problem, keepalive, u_out, device, dtype code)."""
    if _is_torch(F):
        import torch
        tdt = torch.float64 if dtype == "f64" else torch.float32
        if F.dtype != tdt or not F.is_contiguous():
            F = F.to(tdt).contiguous()
        dev = F.device

        def as_dev(x, dt):
            # tensors already in place are used as they are
            if _is_torch(x) and x.dtype == dt and x.device == dev and x.is_contiguous():
                return x
            if not _is_torch(x):
                x = np.asarray(x)
            return torch.as_tensor(x, device=dev).to(dt).contiguous()

        srct = as_dev(src if _is_torch(src) else np.asarray(src, dtype=np.int64).ravel(), torch.int64)
        qt = None if q is None else as_dev(q, torch.float64)
        mt = None if mask is None else as_dev(mask, torch.uint8)
        _check_arrays(F.shape, mt, qt, srct.numel(), u_out, tdt, dev)
        if u_out is None:
            u_out = torch.empty_like(F)
        ny, nx = F.shape
        p = Problem(nx, ny, float(h), F.data_ptr(), None if mt is None else mt.data_ptr(),
                    srct.numel(), srct.data_ptr(), None if qt is None else qt.data_ptr(),
                    u_out.data_ptr())
        return p, (F, srct, qt, mt, u_out), u_out, True
    ndt = np.float64 if dtype == "f64" else np.float32
    F = np.ascontiguousarray(F, dtype=ndt)
    srca = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
    qa = None if q is None else np.ascontiguousarray(np.atleast_1d(q), dtype=np.float64)
    ma = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    _check_arrays(F.shape, ma, qa, len(srca), u_out, np.dtype(ndt), None)
    if u_out is None:
        u_out = np.empty_like(F)
    ny, nx = F.shape
    p = Problem(nx, ny, float(h), F.ctypes.data, None if ma is None else ma.ctypes.data,
                len(srca), srca.ctypes.data, None if qa is None else qa.ctypes.data,
                u_out.ctypes.data)
    return p, (F, srca, qa, ma, u_out), u_out, False


def _stream_of(device: bool):
    if not device:
        return None
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def eik_solve(F, h, src, q=None, mask=None, u_out=None, *, dtype="f64", method="exact",
              cell=0, band=0.0, workers=0, residual_check=False, max_cell_visits=0,
              band_window=0, eager_publish=False, schedule="auto", timeout_ms=0, graph=False,
              residual_tol=0.0, band_cells=0.0):
    """Solves |grad u| F = 1 with u = q on src (see include/eik.h).
    Returns (u, stats dict)."""
    p, keep, u_out, device = _marshal(F, h, src, q, mask, u_out, dtype)
    o = _opts(F64 if dtype == "f64" else F32, method, cell, band, device, _stream_of(device),
              residual_check, workers, max_cell_visits, band_window, eager_publish, schedule,
              timeout_ms, graph, residual_tol, band_cells)
    st = Stats()
    _check(lib.eik_solve(p.nx, p.ny, p.h, p.F, p.mask, p.nsrc, p.src, p.q, p.u_out,
                         ctypes.byref(o), ctypes.byref(st)))
    del keep
    return u_out, st.as_dict()


def eik_solve_batched(problems, *, dtype="f64", method="exact", cell=0, band=0.0, workers=0,
                      residual_check=False, max_cell_visits=0, band_window=0,
                      eager_publish=False, schedule="auto", timeout_ms=0, graph=False,
                      residual_tol=0.0, band_cells=0.0):
    """problems: list of dicts with F, h, src and optional q, mask, u_out.
    Returns (list of u, list of stats dicts)."""
    ps, keeps, outs = [], [], []
    device = None
    for w in problems:
        p, keep, u, dev = _marshal(w["F"], w["h"], w["src"], w.get("q"), w.get("mask"),
                                   w.get("u_out"), dtype)
        if device is None:
            device = dev
        elif device != dev:
            raise ValueError("all problems of a batch must be host or all device arrays")
        ps.append(p)
        keeps.append(keep)
        outs.append(u)
    arr = (Problem * len(ps))(*ps)
    o = _opts(F64 if dtype == "f64" else F32, method, cell, band, device, _stream_of(device),
              residual_check, workers, max_cell_visits, band_window, eager_publish, schedule,
              timeout_ms, graph, residual_tol, band_cells)
    st = (Stats * len(ps))()
    _check(lib.eik_solve_batched(len(ps), arr, ctypes.byref(o), st))
    del keeps
    return outs, [s.as_dict() for s in st]


def eik_sweep(F, h, src, q=None, mask=None, u_out=None, *, dtype="f64", locking=False,
              max_sweeps=0, threshold=0.0):
    """Whole-grid Fast Sweeping (locking=False) or Locking Sweeping with tile
    locks (eik_sweep_solve of include/eik.h).  Returns (u, largest decrease
    per sweep, decreased nodes per sweep, stats dict); the per-sweep arrays
    hold one entry per sweep performed."""
    p, keep, u_out, device = _marshal(F, h, src, q, mask, u_out, dtype)
    o = SweepOpts(F64 if dtype == "f64" else F32, int(bool(locking)), int(max_sweeps),
                  float(threshold), int(device), _stream_of(device))
    cap = int(max_sweeps) if max_sweeps > 0 else 65536
    mx = np.zeros(cap, dtype=np.float64)
    cnt = np.zeros(cap, dtype=np.int64)
    st = SweepStats()
    _check(lib.eik_sweep_solve(p.nx, p.ny, p.h, p.F, p.mask, p.nsrc, p.src, p.q, p.u_out,
                               ctypes.byref(o), mx.ctypes.data, cnt.ctypes.data, ctypes.byref(st)))
    del keep
    k = st.sweeps
    return u_out, mx[:k].copy(), cnt[:k].copy(), {f: getattr(st, f) for f, _ in st._fields_}


def eik_solve3(F, h, src, q=None, mask=None, u_out=None, *, method="exact"):
    """3-D solve (eik_solve3, or eik_fmsm3 with method="fmsm", of
    include/eik.h); F has shape (nz, ny, nx), FP64.  numpy arrays are host
    inputs, torch tensors device inputs.  Returns (u, stats dict)."""
    if method not in ("exact", "fmsm"):
        raise ValueError(f"method {method!r}: 'exact' or 'fmsm'")
    if _is_torch(F):
        import torch
        dev = F.device
        F_ = F.to(torch.float64).contiguous()
        src_ = torch.as_tensor(np.asarray(src, dtype=np.int64).ravel() if not _is_torch(src) else src,
                               device=dev).to(torch.int64).contiguous()
        q_ = None if q is None else torch.as_tensor(q if _is_torch(q) else np.asarray(q),
                                                    device=dev).to(torch.float64).contiguous()
        m_ = None if mask is None else torch.as_tensor(mask if _is_torch(mask) else np.asarray(mask),
                                                       device=dev).to(torch.uint8).contiguous()
        _check_arrays(F_.shape, m_, q_, src_.numel(), u_out, torch.float64, dev)
        u = torch.empty_like(F_) if u_out is None else u_out
        ptr = lambda t: None if t is None else t.data_ptr()
        nsrc = src_.numel()
        device = True
    else:
        F_ = np.ascontiguousarray(F, dtype=np.float64)
        src_ = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
        q_ = None if q is None else np.ascontiguousarray(np.atleast_1d(q), dtype=np.float64)
        m_ = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        _check_arrays(F_.shape, m_, q_, len(src_), u_out, np.dtype(np.float64), None)
        u = np.empty_like(F_) if u_out is None else u_out
        ptr = lambda a: None if a is None else a.ctypes.data
        nsrc = len(src_)
        device = False
    nz, ny, nx = F_.shape
    st = Stats3()
    fn = lib.eik_solve3 if method == "exact" else lib.eik_fmsm3
    _check(fn(nx, ny, nz, float(h), ptr(F_), ptr(m_), nsrc, ptr(src_), ptr(q_), ptr(u),
              int(device), _stream_of(device), ctypes.byref(st)))
    return u, {f: getattr(st, f) for f, _ in st._fields_}


def probe_step_latency(dtype="f64", side=64, sweeps=200) -> float:
    """Seconds per dependent anti-diagonal step of the cell sweep, one wave
    alone (eik_probe_step_latency of include/eik.h)."""
    t = ctypes.c_double()
    _check(lib.eik_probe_step_latency(F64 if dtype == "f64" else F32, int(side), int(sweeps),
                                      ctypes.byref(t)))
    return t.value


class Server:
    """Continuous-batching server (eik_serve_* of include/eik.h).

    submit() takes numpy arrays (host inputs, copied at once) or device
    tensors (read when the request is admitted; kept alive here until the
    result is collected).  Results are host numpy arrays."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, lanes=0, *, dtype="f64",
                 method="exact", cell=0, band=0.0, residual_check=False, device_inputs=False,
                 schedule="auto", max_cell_visits=0, residual_tol=0.0):
        self.dtype = dtype
        o = _opts(F64 if dtype == "f64" else F32, method, cell, band, device_inputs, None,
                  residual_check, 0, max_cell_visits, 0, False, schedule, 0, False, residual_tol)
        cfg = ServeCfg(int(hbm_budget_bytes), int(max_slots), int(lanes), o)
        h = ctypes.c_void_p()
        _check(lib.eik_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, F, h, src, q=None, mask=None) -> int:
        p, keep, _, _ = _marshal(F, h, src, q, mask, None, self.dtype)
        ndt = np.float64 if self.dtype == "f64" else np.float32
        u = np.empty((p.ny, p.nx), dtype=ndt)
        p.u_out = u.ctypes.data
        t = ctypes.c_uint64()
        _check(lib.eik_serve_submit(self._h, ctypes.byref(p), ctypes.byref(t)))
        self._keep[t.value] = (u, keep)
        return t.value

    def _collect(self, rc, ticket, st):
        if rc == EIK_EBUSY:
            return None
        u, _ = self._keep.pop(ticket, (None, None))
        _check(rc)
        return u, st.as_dict()

    def poll(self, ticket):
        """(u, stats) when done, None while pending; raises on failure."""
        st = Stats()
        return self._collect(lib.eik_serve_poll(self._h, ticket, ctypes.byref(st)), ticket, st)

    def wait(self, ticket):
        st = Stats()
        return self._collect(lib.eik_serve_wait(self._h, ticket, ctypes.byref(st)), ticket, st)

    def cancel(self, ticket) -> bool:
        rc = lib.eik_serve_cancel(self._h, ticket)
        if rc == EIK_OK:
            self._keep.pop(ticket, None)
            return True
        if rc == EIK_EBUSY:
            return False
        _check(rc)

    def close(self):
        if self._h:
            _check(lib.eik_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """A batch marshalled once and solved repeatedly (eik_solve_batched);
    with graph=True the library replays the batch's captured launch sequence
    from the second solve on.  problems: dicts with F, h, src and optional q,
    mask, u_out (device tensors, or numpy arrays for host problems)."""

    def __init__(self, problems, *, dtype="f64", method="exact", cell=0, band=0.0, workers=0,
                 residual_check=False, max_cell_visits=0, band_window=0, eager_publish=False,
                 schedule="auto", timeout_ms=0, graph=True, residual_tol=0.0, band_cells=0.0):
        ps, self._keep, self.outputs = [], [], []
        device = None
        for w in problems:
            p, keep, u, dev = _marshal(w["F"], w["h"], w["src"], w.get("q"), w.get("mask"),
                                       w.get("u_out"), dtype)
            if device is None:
                device = dev
            elif device != dev:
                raise ValueError("all problems of a batch must be host or all device arrays")
            ps.append(p)
            self._keep.append(keep)
            self.outputs.append(u)
        self._n = len(ps)
        self._arr = (Problem * self._n)(*ps)
        self._device = device
        self._args = (F64 if dtype == "f64" else F32, method, cell, band, device, residual_check,
                      workers, max_cell_visits, band_window, eager_publish, schedule, timeout_ms,
                      graph, residual_tol, band_cells)
        self._stats = (Stats * self._n)()

    def solve(self, stats=True):
        """Solves the batch into self.outputs; returns the stats dicts, or
        None with stats=False (building 256 dicts takes ~1 ms of Python; the
        last call's statistics stay available through stats())."""
        (dt, method, cell, band, device, resid, workers, mcv, bw, eager, sched, tmo,
         graph, rtol, bcells) = self._args
        o = _opts(dt, method, cell, band, device, _stream_of(device), resid, workers, mcv, bw,
                  eager, sched, tmo, graph, rtol, bcells)
        _check(lib.eik_solve_batched(self._n, self._arr, ctypes.byref(o), self._stats))
        return self.stats() if stats else None

    def stats(self):
        """Statistics of the last solve, one dict per problem."""
        return [s.as_dict() for s in self._stats]
