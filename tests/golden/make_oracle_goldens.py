"""Writes the oracle's whole-solve results at the benchmark's full sizes.

Test infrastructure: this script imports only the CPU oracle (``oracle``)
and the seeded input generators (``paper_1804_04737_amd.lpgen``, random
draws only).  Nothing here comes from the GPU library.  The files it writes
are the expected values of ``tests/test_gpu_fullsize.py`` and
``tests/test_gpu_batch.py``:

  fullsize_<m>x<n>_seed0.npz   one dense LP (generator ``lpgen.dense_lp``),
                               solved to the end from the slack basis
                               (Section 2, Steps 1-5, iterated as in
                               Section 3): status, pivot count, the whole
                               (k, l) pivot sequence, the final basis and the
                               IEEE-754 bit patterns of x, y and z.
  batch1024_seed0.npz          the 1024 LPs of ``lpgen.batch_lps(1024, 32,
                               1024, 0)``: per LP status, pivot count, the
                               bit pattern of z and the SHA-256 of x's bit
                               patterns.

Usage:  python tests/golden/make_oracle_goldens.py [--jobs J] [--only NAME]
The 8192 x 8192 solve (3768 pivots) takes several minutes on one core; the
other solves run beside it in a process pool.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FULLSIZE = [(8192, 8192), (4096, 4096), (8192, 1024), (1024, 8192), (2048, 8192)]
BATCH = (1024, 32, 1024, 0)  # count, smallest and largest m and n, seed


def fullsize_path(m: int, n: int) -> str:
    return os.path.join(HERE, f"fullsize_{m}x{n}_seed0.npz")


def batch_path() -> str:
    return os.path.join(HERE, "batch1024_seed0.npz")


def x_digest(x: np.ndarray) -> bytes:
    """SHA-256 of the little-endian IEEE-754 bit patterns of x."""
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).digest()


def _fullsize(shape):
    import oracle
    from paper_1804_04737_amd import lpgen
    m, n = shape
    A, b, c = lpgen.dense_lp(m, n, 0)
    t0 = time.perf_counter()
    r = oracle.solve(A, b, c)
    el = time.perf_counter() - t0
    np.savez_compressed(
        fullsize_path(m, n),
        m=m, n=n, seed=0, status=r.status, iterations=r.iterations,
        trace=r.trace.astype(np.int32), basis=r.basis.astype(np.int32),
        x_bits=r.x.view(np.int64), y_bits=r.y.view(np.int64),
        obj_bits=np.array([r.obj]).view(np.int64),
        provenance=np.array("oracle.solve(*lpgen.dense_lp(m, n, 0)), default eps and iteration cap; "
                            "written by tests/golden/make_oracle_goldens.py"))
    return f"{m}x{n}: {r.status_name} after {r.iterations} pivots, z = {r.obj!r} ({el:.1f} s)"


def _batch_part(lo_hi):
    import oracle
    from paper_1804_04737_amd import lpgen
    lo, hi = lo_hi
    count, smin, smax, seed = BATCH
    out = []
    for i in range(lo, hi):
        A, b, c = lpgen.batch_lp(i, count, smin, smax, seed)
        r = oracle.solve(A, b, c)
        out.append((i, r.status, r.iterations, np.array([r.obj]).view(np.int64)[0], x_digest(r.x)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", default="", help="fullsize_MxN or batch (default: everything)")
    args = ap.parse_args()
    import oracle
    oracle.build()  # the same C source the tests load
    todo_full = [s for s in FULLSIZE if args.only in ("", f"fullsize_{s[0]}x{s[1]}")]
    do_batch = args.only in ("", "batch")
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        futs = [ex.submit(_fullsize, s) for s in todo_full]
        parts = []
        if do_batch:
            count = BATCH[0]
            step = 16
            parts = [ex.submit(_batch_part, (lo, min(count, lo + step))) for lo in range(0, count, step)]
        if parts:
            rows = sorted(r for p in parts for r in p.result())
            np.savez_compressed(
                batch_path(),
                count=BATCH[0], lo=BATCH[1], hi=BATCH[2], seed=BATCH[3],
                status=np.array([r[1] for r in rows], np.int32),
                iterations=np.array([r[2] for r in rows], np.int64),
                obj_bits=np.array([r[3] for r in rows], np.int64),
                x_sha256=np.frombuffer(b"".join(r[4] for r in rows), np.uint8).reshape(-1, 32),
                provenance=np.array("oracle.solve of each LP of lpgen.batch_lps(1024, 32, 1024, 0); "
                                    "written by tests/golden/make_oracle_goldens.py"))
            print(f"batch: {len(rows)} LPs, {int(sum(r[2] for r in rows))} pivots", flush=True)
        for f in futs:
            print(f.result(), flush=True)


if __name__ == "__main__":
    main()
