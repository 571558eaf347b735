"""Reference oracle for the dense-tableau simplex (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it, and it shares no
code with the HIP path: the arithmetic lives in ``tableau_simplex.c``
(standard simplex, Section 2 of Coutinho et al., Steps 1-5, iterated as in
Section 3), this module only marshals numpy arrays through ctypes.  The same
source is also built with OpenMP (``liboracle_omp.so``: Step 5's rows in
parallel threads, every value unchanged) for the benchmark's multi-core
baseline.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tableau_simplex.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OPTIMAL, UNBOUNDED, ITERATION_LIMIT, INFEASIBLE_START, NUMERICAL = range(5)
STATUS_NAMES = ("OPTIMAL", "UNBOUNDED", "ITERATION_LIMIT", "INFEASIBLE_START", "NUMERICAL")

# -ffp-contract=off: the only fused multiply-add is the explicit fma() call.
CFLAGS = ["-O3", "-mavx2", "-std=c11", "-mfma", "-ffp-contract=off", "-fno-math-errno",
          "-fno-fast-math", "-shared", "-fPIC"]


def build(src: str = _SRC, out: str = _LIB, extra_flags=()) -> str:
    """Compile the C oracle into a shared library (always recompiles).  The
    file is replaced atomically, so processes that loaded the old one keep
    it."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_omp() -> str:
    """The same source with OpenMP threads in Step 5 (liboracle_omp.so)."""
    return build(out=_LIB_OMP, extra_flags=("-fopenmp",))


_lib = None


def _load(path: str = _LIB):
    global _lib
    if _lib is not None and path == _LIB:
        return _lib
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    f = lib.oracle_solve
    P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    f.restype = ctypes.c_int
    f.argtypes = [I64, I64, P, P, P, D, D, I64, P, P, P, P, P, P, I64, P]
    if hasattr(lib, "oracle_solve_tableau"):
        lib.oracle_solve_tableau.restype = ctypes.c_int
        lib.oracle_solve_tableau.argtypes = [I64, I64, P, P, D, D, I64, P, P, I64]
        lib.oracle_pivot.restype = ctypes.c_int
        lib.oracle_pivot.argtypes = [I64, I64, P, I64, I64]
        lib.oracle_price_out.restype = ctypes.c_int
        lib.oracle_price_out.argtypes = [I64, I64, P, P]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
    if path == _LIB:
        _lib = lib
    return lib


def load_omp():
    """The OpenMP build (built on first use)."""
    if not os.path.exists(_LIB_OMP):
        build_omp()
    return _load(_LIB_OMP)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    status: int
    x: np.ndarray
    obj: float
    y: np.ndarray
    iterations: int
    basis: np.ndarray
    trace: np.ndarray        # (iterations_recorded, 2): entering column k, leaving row l
    tableau: np.ndarray | None  # (m+1, n+m+1) final tableau if requested

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def solve(A, b, c, *, eps_d: float = 1e-9, eps_p: float = 1e-9, max_iter: int | None = None,
          want_tableau: bool = False, trace_cap: int | None = None, lib_path: str | None = None
          ) -> OracleResult:
    """Run the C oracle on host arrays (converted to contiguous float64)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1)
    m, n = A.shape
    if b.shape[0] != m or c.shape[0] != n:
        raise ValueError("shape mismatch between A, b and c")
    if max_iter is None:
        max_iter = 50 * (m + n)
    if trace_cap is None:
        trace_cap = min(max_iter, 1 << 20)
    lib = _load(lib_path or _LIB)
    x = np.zeros(n)
    y = np.zeros(m)
    obj = np.zeros(1)
    iters = np.zeros(1, dtype=np.int64)
    basis = np.zeros(m, dtype=np.int64)
    trace = np.zeros(2 * max(trace_cap, 1), dtype=np.int32)
    tab = np.zeros((m + 1, n + m + 1)) if want_tableau else None
    st = lib.oracle_solve(m, n, _ptr(A), _ptr(b), _ptr(c), eps_d, eps_p, int(max_iter),
                          _ptr(x), _ptr(obj), _ptr(y), _ptr(iters), _ptr(basis), _ptr(trace),
                          int(trace_cap), _ptr(tab))
    if st < 0:
        raise ValueError(f"oracle_solve rejected its arguments (code {st})")
    it = int(iters[0])
    rec = min(it, trace_cap)
    return OracleResult(st, x, float(obj[0]), y, it, basis,
                        trace[: 2 * rec].reshape(rec, 2).copy(), tab)


@dataclass
class TableauResult:
    status: int
    tableau: np.ndarray     # (m+1, ncols+1) final tableau
    basis: np.ndarray       # (m,) int64 variable (column) of each row
    iterations: int
    trace: np.ndarray       # (iterations_recorded, 2): entering column k, leaving row l

    @property
    def x(self) -> np.ndarray:
        """Value of every column's variable: its row's RHS if basic, else 0."""
        T = self.tableau
        x = np.zeros(T.shape[1] - 1)
        for i, v in enumerate(self.basis):
            x[v] = T[i, -1]
        return x

    @property
    def obj(self) -> float:
        return float(self.tableau[-1, -1])


def solve_tableau(T, basis, *, eps_d: float = 1e-9, eps_p: float = 1e-9, max_iter: int | None = None,
                  trace_cap: int | None = None, lib_path: str | None = None) -> TableauResult:
    """Steps 2-5 from the basic tableau T ((m+1) x (ncols+1), RHS last,
    objective row last) with basis[i] the column of row i's basic variable.
    T and basis are copied, not changed."""
    T = np.array(T, dtype=np.float64, order="C", copy=True)
    basis = np.array(basis, dtype=np.int64, copy=True).reshape(-1)
    m, ncols = T.shape[0] - 1, T.shape[1] - 1
    if basis.shape[0] != m:
        raise ValueError("basis must have one entry per constraint row")
    if max_iter is None:
        max_iter = 50 * ncols
    if trace_cap is None:
        trace_cap = min(max_iter, 1 << 20)
    lib = _load(lib_path or _LIB)
    iters = np.zeros(1, dtype=np.int64)
    trace = np.zeros(2 * max(trace_cap, 1), dtype=np.int32)
    st = lib.oracle_solve_tableau(m, ncols, _ptr(T), _ptr(basis), eps_d, eps_p, int(max_iter), _ptr(iters),
                                  _ptr(trace), int(trace_cap))
    if st < 0:
        raise ValueError(f"oracle_solve_tableau rejected its arguments (code {st})")
    it = int(iters[0])
    rec = min(it, trace_cap)
    return TableauResult(st, T, basis, it, trace[: 2 * rec].reshape(rec, 2).copy())


def pivot(T, l: int, k: int, lib_path: str | None = None) -> None:
    """Steps 4-5 on the element (l, k) of T (float64, C order), in place."""
    assert T.dtype == np.float64 and T.flags.c_contiguous
    rc = _load(lib_path or _LIB).oracle_pivot(T.shape[0] - 1, T.shape[1] - 1, _ptr(T), int(l), int(k))
    if rc < 0:
        raise ValueError("oracle_pivot rejected its arguments")


def price_out(T, basis, lib_path: str | None = None) -> None:
    """Eliminates the basic columns from the objective row of T, in place."""
    assert T.dtype == np.float64 and T.flags.c_contiguous
    basis = np.ascontiguousarray(basis, dtype=np.int64)
    rc = _load(lib_path or _LIB).oracle_price_out(T.shape[0] - 1, T.shape[1] - 1, _ptr(T), _ptr(basis))
    if rc < 0:
        raise ValueError("oracle_price_out rejected its arguments")
