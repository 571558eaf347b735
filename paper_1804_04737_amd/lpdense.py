"""Thin Python binding of the lpdense C ABI (include/lpdense.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the in-tree `liblpdense.so`.  PyTorch supplies device memory and the current
HIP stream.  There is no CPU fallback: if the library is missing or cannot be
loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblpdense.so")

OPTIMAL, UNBOUNDED, ITERATION_LIMIT, INFEASIBLE_START, NUMERICAL, DEVICE_TIMEOUT, INFEASIBLE = range(7)
STATUS_NAMES = ("OPTIMAL", "UNBOUNDED", "ITERATION_LIMIT", "INFEASIBLE_START", "NUMERICAL",
                "DEVICE_TIMEOUT", "INFEASIBLE")
ROW_LE, ROW_EQ, ROW_GE = 0, 1, 2
SCHED_AUTO, SCHED_WORKGROUP, SCHED_GRID, SCHED_GRID_CONDENSED, SCHED_GRID_PAIRED = 0, 1, 2, 3, 4
SCHED_GRID_CONDENSED_PAIRED = 5

# Exported symbols, as declared in include/lpdense.h.
EXPORTS = ("lp_solve_dense", "lp_solve_dense_ex", "lp_solve_dense_noalloc", "lp_solve_tableau", "lp_solve_batch", "lp_solve_general", "lpd_server_create",
           "lpd_server_submit", "lpd_server_poll", "lpd_server_get_stats", "lpd_server_destroy",
           "lpd_workspace_bytes", "lpd_error_string", "lpd_status_string", "lpd_version")

_P = ctypes.c_void_p
_I64 = ctypes.c_int64


class Problem(ctypes.Structure):
    _fields_ = [("m", _I64), ("n", _I64), ("A", _P), ("b", _P), ("c", _P)]


class Options(ctypes.Structure):
    _fields_ = [("eps_d", ctypes.c_double), ("eps_p", ctypes.c_double), ("max_iter", _I64),
                ("schedule", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("watchdog_us", _I64)]


class Outputs(ctypes.Structure):
    _fields_ = [("x", _P), ("obj", _P), ("status", _P), ("y", _P), ("iterations", _P),
                ("trace", _P), ("trace_cap", _I64), ("basis", _P), ("tableau", _P),
                ("phase_ticks", _P), ("phase_cap", _I64)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("eps_d", ctypes.c_double), ("eps_p", ctypes.c_double), ("max_iter", _I64),
                ("team_size", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("team_min_bytes", _I64), ("iterations", _P), ("team_bytes_per_wg", _I64),
                ("wave_slots", ctypes.c_int32), ("full_tableau", ctypes.c_int32)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("eps_d", ctypes.c_double), ("eps_p", ctypes.c_double), ("max_iter", _I64),
                ("pivots_per_epoch", _I64), ("max_resident", ctypes.c_int32),
                ("full_tableau", ctypes.c_int32), ("team_min_bytes", _I64), ("team_bytes_per_wg", _I64),
                ("epoch_bytes_per_wg", _I64), ("admit_bytes_per_round", _I64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", _I64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("obj", ctypes.c_double), ("iterations", _I64), ("m", _I64), ("n", _I64),
                ("x", _P), ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _I64), ("completed", _I64), ("epochs", _I64), ("resident", _I64),
                ("waiting", _I64), ("used_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("copy_bytes", ctypes.c_uint64),
                ("kernel_seconds", ctypes.c_double), ("admit_host_seconds", ctypes.c_double)]


class LpdError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed: {error_string(code)} ({code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1804_04737_amd.build`")
    lib = ctypes.CDLL(path)
    lib.lp_solve_dense.restype = ctypes.c_int
    lib.lp_solve_dense.argtypes = [_I64, _I64, _P, _P, _P, _P, _P, _P, _P]
    lib.lp_solve_dense_ex.restype = ctypes.c_int
    lib.lp_solve_dense_ex.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                      ctypes.POINTER(Outputs), _P]
    lib.lp_solve_dense_noalloc.restype = ctypes.c_int
    lib.lp_solve_dense_noalloc.argtypes = lib.lp_solve_dense_ex.argtypes
    lib.lp_solve_tableau.restype = ctypes.c_int
    lib.lp_solve_tableau.argtypes = [_I64, _I64, _P, _P, ctypes.POINTER(Options), ctypes.POINTER(Outputs), _P]
    lib.lp_solve_batch.restype = ctypes.c_int
    lib.lp_solve_batch.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                   ctypes.POINTER(BatchOptions), _P]
    lib.lp_solve_general.restype = ctypes.c_int
    lib.lp_solve_general.argtypes = [_I64, _I64, _P, _P, _P, _P, ctypes.POINTER(Options), _P, _P, _P, _P, _P]
    lib.lpd_server_create.restype = _P
    lib.lpd_server_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ServerOptions)]
    lib.lpd_server_submit.restype = _I64
    lib.lpd_server_submit.argtypes = [_P, _I64, _I64, _P, _P, _P, _P]
    lib.lpd_server_poll.restype = ctypes.c_int
    lib.lpd_server_poll.argtypes = [_P, ctypes.POINTER(Completion), ctypes.c_int]
    lib.lpd_server_get_stats.restype = ctypes.c_int
    lib.lpd_server_get_stats.argtypes = [_P, ctypes.POINTER(ServerStats)]
    lib.lpd_server_destroy.restype = None
    lib.lpd_server_destroy.argtypes = [_P]
    lib.lpd_workspace_bytes.restype = ctypes.c_uint64
    lib.lpd_workspace_bytes.argtypes = [_I64, _I64]
    lib.lpd_error_string.restype = ctypes.c_char_p
    lib.lpd_error_string.argtypes = [ctypes.c_int]
    lib.lpd_status_string.restype = ctypes.c_char_p
    lib.lpd_status_string.argtypes = [ctypes.c_int32]
    lib.lpd_version.restype = ctypes.c_int
    lib.lpd_version.argtypes = []
    _lib = lib
    return lib


def error_string(code: int) -> str:
    return load().lpd_error_string(int(code)).decode()


def workspace_bytes(m: int, n: int) -> int:
    return int(load().lpd_workspace_bytes(int(m), int(n)))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(name, t, dtype, numel):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")


def solve_dense(A, b, c, x=None, obj=None, status=None, stream=None):
    """lp_solve_dense on device tensors; returns (x, obj, status) device tensors.

    Asynchronous on `stream` (default: torch's current stream)."""
    import torch
    m, n = A.shape
    _check_dev("A", A, torch.float64, m * n)
    _check_dev("b", b, torch.float64, m)
    _check_dev("c", c, torch.float64, n)
    dev = A.device
    x = torch.empty(n, dtype=torch.float64, device=dev) if x is None else x
    obj = torch.empty(1, dtype=torch.float64, device=dev) if obj is None else obj
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    rc = load().lp_solve_dense(m, n, _ptr(A), _ptr(b), _ptr(c), _ptr(x), _ptr(obj), _ptr(status),
                               _stream_handle(stream))
    if rc != 0:
        raise LpdError(rc, "lp_solve_dense")
    return x, obj, status


@dataclass
class DenseResult:
    x: "object"
    obj: "object"
    status: "object"
    y: "object"
    iterations: "object"
    trace: "object"
    basis: "object"
    tableau: "object"
    phase_ticks: "object" = None


def solve_dense_ex(A, b, c, *, eps_d: float = 0.0, eps_p: float = 0.0, max_iter: int = -1,
                   schedule: int = SCHED_AUTO, grid_blocks: int = 0, want_y: bool = True,
                   trace_cap: int = 0, want_basis: bool = False, want_tableau: bool = False,
                   phase_cap: int = 0, stream=None, noalloc: bool = False,
                   watchdog_us: int = 0) -> DenseResult:
    """lp_solve_dense_ex on device tensors; outputs are freshly allocated
    device tensors (asynchronous: synchronise the stream before reading).
    noalloc=True calls lp_solve_dense_noalloc instead (the library's fixed
    workspace, no device allocation inside the call)."""
    import torch
    m, n = A.shape
    _check_dev("A", A, torch.float64, m * n)
    _check_dev("b", b, torch.float64, m)
    _check_dev("c", c, torch.float64, n)
    dev = A.device
    f64, i32, i64 = torch.float64, torch.int32, torch.int64
    res = DenseResult(
        x=torch.empty(n, dtype=f64, device=dev),
        obj=torch.empty(1, dtype=f64, device=dev),
        status=torch.empty(1, dtype=i32, device=dev),
        y=torch.empty(m, dtype=f64, device=dev) if want_y else None,
        iterations=torch.empty(1, dtype=i64, device=dev),
        trace=torch.empty((max(trace_cap, 0), 2), dtype=i32, device=dev) if trace_cap > 0 else None,
        basis=torch.empty(m, dtype=i64, device=dev) if want_basis else None,
        tableau=torch.empty((m + 1, n + m + 1), dtype=f64, device=dev) if want_tableau else None,
        phase_ticks=torch.zeros((phase_cap, 8), dtype=i64, device=dev) if phase_cap > 0 else None,
    )
    prob = Problem(m, n, A.data_ptr(), b.data_ptr(), c.data_ptr())
    opts = Options(float(eps_d), float(eps_p), int(max_iter), int(schedule), int(grid_blocks), int(watchdog_us))
    outs = Outputs(res.x.data_ptr(), res.obj.data_ptr(), res.status.data_ptr(),
                   res.y.data_ptr() if res.y is not None else None,
                   res.iterations.data_ptr(),
                   res.trace.data_ptr() if res.trace is not None else None,
                   int(max(trace_cap, 0)),
                   res.basis.data_ptr() if res.basis is not None else None,
                   res.tableau.data_ptr() if res.tableau is not None else None,
                   res.phase_ticks.data_ptr() if res.phase_ticks is not None else None,
                   int(max(phase_cap, 0)))
    fn = load().lp_solve_dense_noalloc if noalloc else load().lp_solve_dense_ex
    rc = fn(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(outs), _stream_handle(stream))
    if rc != 0:
        raise LpdError(rc, "lp_solve_dense_noalloc" if noalloc else "lp_solve_dense_ex")
    return res


def solve_tableau(T0, basis0, *, eps_d: float = 0.0, eps_p: float = 0.0, max_iter: int = -1,
                  schedule: int = SCHED_AUTO, grid_blocks: int = 0, trace_cap: int = 0,
                  want_basis: bool = False, want_tableau: bool = False, stream=None) -> DenseResult:
    """lp_solve_tableau: Steps 2-5 from the basic tableau T0 (a (m+1) x
    (ncols+1) device tensor, RHS last, objective row last) whose row i has
    basic variable basis0[i] (host sequence of m column indices).  Outputs
    are fresh device tensors; x has ncols entries (asynchronous)."""
    import numpy as np
    import torch
    if T0.dim() != 2:
        raise ValueError("T0 must be a matrix")
    m, ncols = T0.shape[0] - 1, T0.shape[1] - 1
    _check_dev("T0", T0, torch.float64, (m + 1) * (ncols + 1))
    b0 = np.ascontiguousarray(np.asarray(basis0, dtype=np.int64))
    if b0.shape != (m,):
        raise ValueError("basis0 must have one entry per constraint row")
    dev = T0.device
    f64, i32, i64 = torch.float64, torch.int32, torch.int64
    res = DenseResult(
        x=torch.empty(ncols, dtype=f64, device=dev),
        obj=torch.empty(1, dtype=f64, device=dev),
        status=torch.empty(1, dtype=i32, device=dev),
        y=None,
        iterations=torch.empty(1, dtype=i64, device=dev),
        trace=torch.empty((max(trace_cap, 0), 2), dtype=i32, device=dev) if trace_cap > 0 else None,
        basis=torch.empty(m, dtype=i64, device=dev) if want_basis else None,
        tableau=torch.empty((m + 1, ncols + 1), dtype=f64, device=dev) if want_tableau else None,
    )
    opts = Options(float(eps_d), float(eps_p), int(max_iter), int(schedule), int(grid_blocks))
    outs = Outputs(res.x.data_ptr(), res.obj.data_ptr(), res.status.data_ptr(), None,
                   res.iterations.data_ptr(),
                   res.trace.data_ptr() if res.trace is not None else None, int(max(trace_cap, 0)),
                   res.basis.data_ptr() if res.basis is not None else None,
                   res.tableau.data_ptr() if res.tableau is not None else None, None, 0)
    rc = load().lp_solve_tableau(m, ncols, T0.data_ptr(), b0.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(opts), ctypes.byref(outs), _stream_handle(stream))
    if rc != 0:
        raise LpdError(rc, "lp_solve_tableau")
    return res


@dataclass
class PackedBatch:
    """A batch of LPs packed into device arrays, with host offset tables, and
    the device outputs lp_solve_batch fills."""
    m: "object"        # host int64 arrays
    n: "object"
    A_off: "object"
    b_off: "object"
    c_off: "object"
    x_off: "object"
    A: "object"        # device float64 packs
    b: "object"
    c: "object"
    x: "object"
    obj: "object"
    status: "object"
    iterations: "object"

    @property
    def count(self) -> int:
        return len(self.m)

    def x_of(self, i):
        return self.x[int(self.x_off[i]): int(self.x_off[i]) + int(self.n[i])]


def pack_batch(lps, device="cuda") -> PackedBatch:
    """Pack host (A, b, c) numpy triples into device arrays (one copy each)."""
    import numpy as np
    import torch
    m = np.array([a.shape[0] for a, _, _ in lps], dtype=np.int64)
    n = np.array([a.shape[1] for a, _, _ in lps], dtype=np.int64)
    def offs(sizes):
        o = np.zeros(len(sizes), dtype=np.int64)
        o[1:] = np.cumsum(sizes)[:-1]
        return o
    A_off, b_off, c_off = offs(m * n), offs(m), offs(n)
    A = np.concatenate([np.ascontiguousarray(a, dtype=np.float64).ravel() for a, _, _ in lps])
    b = np.concatenate([np.asarray(bb, dtype=np.float64) for _, bb, _ in lps])
    c = np.concatenate([np.asarray(cc, dtype=np.float64) for _, _, cc in lps])
    dev = torch.device(device)
    cnt = len(lps)
    return PackedBatch(m, n, A_off, b_off, c_off, c_off.copy(),
                       torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev), torch.from_numpy(c).to(dev),
                       torch.empty(int(n.sum()), dtype=torch.float64, device=dev),
                       torch.empty(cnt, dtype=torch.float64, device=dev),
                       torch.empty(cnt, dtype=torch.int32, device=dev),
                       torch.empty(cnt, dtype=torch.int64, device=dev))


def solve_batch(pb: PackedBatch, *, eps_d: float = 0.0, eps_p: float = 0.0, max_iter: int = -1,
                team_size: int = 0, team_min_bytes: int = 0, team_bytes_per_wg: int = 0,
                wave_slots: int = 0, full_tableau: bool = False, grid_blocks: int = 0,
                stream=None) -> PackedBatch:
    """lp_solve_batch on a PackedBatch (asynchronous; outputs land in pb)."""
    import numpy as np
    def hp(a):
        return a.ctypes.data_as(ctypes.c_void_p)
    opts = BatchOptions(float(eps_d), float(eps_p), int(max_iter), int(team_size), int(grid_blocks),
                        int(team_min_bytes), pb.iterations.data_ptr(), int(team_bytes_per_wg),
                        int(wave_slots), int(bool(full_tableau)))
    m = np.ascontiguousarray(pb.m, dtype=np.int64)
    n = np.ascontiguousarray(pb.n, dtype=np.int64)
    rc = load().lp_solve_batch(pb.count, hp(m), hp(n), pb.A.data_ptr(), hp(pb.A_off), pb.b.data_ptr(),
                               hp(pb.b_off), pb.c.data_ptr(), hp(pb.c_off), pb.x.data_ptr(), hp(pb.x_off),
                               pb.obj.data_ptr(), pb.status.data_ptr(), ctypes.byref(opts),
                               _stream_handle(stream))
    if rc != 0:
        raise LpdError(rc, "lp_solve_batch")
    return pb


@dataclass
class Served:
    """One finished request of a Server."""
    id: int
    status: int
    obj: float
    iterations: int
    x: "object"          # numpy float64 array (n)
    t_arrive: float      # seconds since the server started
    t_admit: float
    t_done: float
    m: int = 0
    n: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class Server:
    """lpd_server_* : continuous batching of LPs submitted from the host.

    submit() takes host numpy arrays (kept alive here until the request
    completes) and returns the request id; poll() returns the requests that
    finished since the last call."""

    def __init__(self, budget_bytes: int, *, device: int = 0, pivots_per_epoch: int = 0,
                 max_resident: int = 0, eps_d: float = 0.0, eps_p: float = 0.0, max_iter: int = 0,
                 team_min_bytes: int = 0, team_bytes_per_wg: int = 0, epoch_bytes_per_wg: int = 0,
                 admit_bytes_per_round: int = 0, full_tableau: bool = False):
        opts = ServerOptions(float(eps_d), float(eps_p), int(max_iter), int(pivots_per_epoch),
                             int(max_resident), int(bool(full_tableau)), int(team_min_bytes),
                             int(team_bytes_per_wg),
                             int(epoch_bytes_per_wg), int(admit_bytes_per_round))
        self._lib = load()
        h = self._lib.lpd_server_create(int(device), int(budget_bytes), ctypes.byref(opts))
        if not h:
            raise RuntimeError("lpd_server_create failed (no usable gfx950 device or out of memory)")
        self._h = ctypes.c_void_p(h)
        self._live = {}
        self._buf = (Completion * 256)()

    def submit(self, A, b, c) -> int:
        import numpy as np
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        m, n = A.shape
        if b.shape != (m,) or c.shape != (n,):
            raise ValueError("b must have m entries and c n entries")
        x = np.empty(n, dtype=np.float64)
        def hp(a):
            return a.ctypes.data_as(ctypes.c_void_p)
        rid = int(self._lib.lpd_server_submit(self._h, m, n, hp(A), hp(b), hp(c), hp(x)))
        if rid < 0:
            raise LpdError(rid, "lpd_server_submit")
        self._live[rid] = (A, b, c, x)
        return rid

    def poll(self):
        out = []
        while True:
            k = self._lib.lpd_server_poll(self._h, self._buf, len(self._buf))
            if k < 0:
                raise LpdError(k, "lpd_server_poll")
            for i in range(k):
                cp = self._buf[i]
                _, _, _, x = self._live.pop(int(cp.id))
                out.append(Served(int(cp.id), int(cp.status), float(cp.obj), int(cp.iterations), x,
                                  float(cp.t_arrive), float(cp.t_admit), float(cp.t_done),
                                  int(cp.m), int(cp.n)))
            if k < len(self._buf):
                return out

    def stats(self) -> ServerStats:
        st = ServerStats()
        rc = self._lib.lpd_server_get_stats(self._h, ctypes.byref(st))
        if rc != 0:
            raise LpdError(rc, "lpd_server_get_stats")
        return st

    @property
    def outstanding(self) -> int:
        return len(self._live)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lpd_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GeneralResult:
    x: "object"
    obj: "object"
    status: "object"
    iterations: "object"


def solve_general(A, b, c, sense=None, *, eps_d: float = 0.0, eps_p: float = 0.0, max_iter: int = -1,
                  schedule: int = SCHED_AUTO, grid_blocks: int = 0, stream=None) -> GeneralResult:
    """lp_solve_general on device tensors (two-phase method; rows <=, =, >=
    given by `sense`, a sequence of ROW_LE / ROW_EQ / ROW_GE, default all <=).
    Synchronous: returns device tensors that are ready."""
    import numpy as np
    import torch
    m, n = A.shape
    _check_dev("A", A, torch.float64, m * n)
    _check_dev("b", b, torch.float64, m)
    _check_dev("c", c, torch.float64, n)
    dev = A.device
    res = GeneralResult(torch.empty(n, dtype=torch.float64, device=dev),
                        torch.empty(1, dtype=torch.float64, device=dev),
                        torch.empty(1, dtype=torch.int32, device=dev),
                        torch.empty(1, dtype=torch.int64, device=dev))
    sn = None
    if sense is not None:
        sn = np.ascontiguousarray(np.asarray(sense, dtype=np.int8))
        if sn.shape != (m,):
            raise ValueError("sense must have one entry per row")
    opts = Options(float(eps_d), float(eps_p), int(max_iter), int(schedule), int(grid_blocks))
    rc = load().lp_solve_general(m, n, A.data_ptr(), b.data_ptr(), c.data_ptr(),
                                 None if sn is None else sn.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(opts), res.x.data_ptr(), res.obj.data_ptr(),
                                 res.status.data_ptr(), res.iterations.data_ptr(), _stream_handle(stream))
    if rc != 0:
        raise LpdError(rc, "lp_solve_general")
    return res
