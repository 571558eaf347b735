"""Reference oracle for the dense-tableau simplex (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it, and it shares no
code with the HIP path: the arithmetic lives in ``tableau_simplex.c``
(standard simplex, Section 2 of Coutinho et al., Steps 1-5, iterated as in
Section 3), this module only marshals numpy arrays through ctypes.
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

OPTIMAL, UNBOUNDED, ITERATION_LIMIT, INFEASIBLE_START, NUMERICAL = range(5)
STATUS_NAMES = ("OPTIMAL", "UNBOUNDED", "ITERATION_LIMIT", "INFEASIBLE_START", "NUMERICAL")

# -ffp-contract=off: the only fused multiply-add is the explicit fma() call.
CFLAGS = ["-O3", "-mavx2", "-std=c11", "-mfma", "-ffp-contract=off", "-fno-math-errno",
          "-fno-fast-math", "-shared", "-fPIC"]


def build(src: str = _SRC, out: str = _LIB, extra_flags=()) -> str:
    """Compile the C oracle into a shared library (always recompiles)."""
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


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
    P = ctypes.c_void_p
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                  ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64, P]
    if path == _LIB:
        _lib = lib
    return lib


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
