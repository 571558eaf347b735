"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default grid: one 1024-thread workgroup per CU).

  * The whole solve of every full-size LP (8192 x 8192 with its 3768 pivots,
    4096 x 4096, 8192 x 1024, 1024 x 8192, 2048 x 8192; generator seed 0) is
    compared with the oracle's, on all four grid schedules: status, pivot
    count, every (k, l) of the pivot sequence, the final basis and the bits of
    x, y and z.  The oracle's results are stored in tests/golden/ by
    tests/golden/make_oracle_goldens.py, which runs only the CPU oracle (the
    8192 x 8192 solve takes minutes on the CPU).  The GPU solution must also
    be primal and dual feasible with a zero duality gap within 1e-9.
  * The first K pivots are compared element by element: the GPU and the
    oracle both run with max_iter = K and return their whole tableaux; sampled
    rows (plus the objective row and every row that was a pivot row) and the
    whole right-hand side must agree bit for bit.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests import lp_checks
from tests.gpu_util import announce, bits, gpu_solve

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SHAPES = [(8192, 8192), (4096, 4096), (8192, 1024), (1024, 8192), (2048, 8192)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_first_pivots_bitwise(m, n):
    A, b, c = lpgen.dense_lp(m, n, 0)
    K = 3
    announce(f"full size {m}x{n}: first {K} pivots with tableau")
    ref = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    rng = np.random.default_rng(m * 7 + n)
    rows = np.unique(np.concatenate([rng.integers(0, m, 64), ref.trace[:, 1], [m]]))
    for schedule in (lpdense.SCHED_AUTO, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED,
                     lpdense.SCHED_GRID_CONDENSED_PAIRED):
        g = gpu_solve(A, b, c, max_iter=K, want_tableau=True, schedule=schedule)
        assert g.status == ref.status == oracle.ITERATION_LIMIT
        assert np.array_equal(g.trace, ref.trace)
        assert np.array_equal(bits(g.tableau[rows]), bits(ref.tableau[rows]))
        assert np.array_equal(bits(g.tableau[:, -1]), bits(ref.tableau[:, -1]))  # whole RHS column
        assert np.array_equal(bits(g.x), bits(ref.x)) and np.array_equal(bits(g.y), bits(ref.y))
        del g


SCHEDULES = [(lpdense.SCHED_AUTO, "grid"), (lpdense.SCHED_GRID_CONDENSED, "condensed"),
             (lpdense.SCHED_GRID_PAIRED, "paired"), (lpdense.SCHED_GRID_CONDENSED_PAIRED, "condensed_paired")]


def _golden(m, n):
    path = os.path.join(GOLDEN, f"fullsize_{m}x{n}_seed0.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("m,n", SHAPES)
def test_full_solve_equals_oracle(m, n):
    A, b, c = lpgen.dense_lp(m, n, 0)
    ref = _golden(m, n)
    assert int(ref["m"]) == m and int(ref["n"]) == n and int(ref["status"]) == oracle.OPTIMAL
    K = int(ref["iterations"])
    for schedule, name in SCHEDULES:
        announce(f"full size {m}x{n}: complete solve, {name} schedule, against the oracle's {K} pivots")
        g = gpu_solve(A, b, c, trace_cap=50 * (m + n), schedule=schedule)
        assert g.status == int(ref["status"]), (name, g.status)
        assert g.iterations == K, (name, g.iterations, K)
        if not np.array_equal(g.trace, ref["trace"]):
            bad = int(np.argmax(np.any(g.trace != ref["trace"], axis=1)))
            raise AssertionError(f"{name}: pivot {bad} differs: gpu {g.trace[bad]} oracle {ref['trace'][bad]}")
        assert np.array_equal(g.basis.astype(np.int64), ref["basis"].astype(np.int64)), name
        assert np.array_equal(bits(g.x), ref["x_bits"]), name
        assert np.array_equal(bits(g.y), ref["y_bits"]), name
        assert bits([g.obj])[0] == int(ref["obj_bits"][0]), name
        if schedule == lpdense.SCHED_AUTO:
            # Properties that hold at any size, from the original data.
            rp, rd, gap = lp_checks.residuals(A, b, c, g.x, g.y)
            assert rp <= 1e-9 and rd <= 1e-9 and gap <= 1e-9, (rp, rd, gap)
            assert lp_checks.complementary_slackness(A, b, c, g.x, g.y) <= 1e-9
        del g
