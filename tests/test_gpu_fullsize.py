"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default grid: one 1024-thread workgroup per CU).

The oracle cannot run thousands of pivots at 8192 x 8192 inside a test, so:
  * the first K pivots are compared exactly: the GPU and the oracle both run
    with max_iter = K and return their whole tableaux; sampled rows (plus the
    objective row and every row that was a pivot row) must agree bit for bit;
  * the full GPU solve must reproduce the oracle's first K pivots in its
    trace, end OPTIMAL, and satisfy properties that hold at any size: primal
    and dual feasibility and a zero duality gap within 1e-9, and
    complementary slackness;
  * the condensed-tableau schedule must give the same bits as the full one
    (first K pivots against the oracle, whole solve against the full path).
"""
import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests import lp_checks
from tests.gpu_util import announce, bits, gpu_solve

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("m,n", SHAPES)
def test_full_solve_properties(m, n):
    A, b, c = lpgen.dense_lp(m, n, 0)
    K = 3
    announce(f"full size {m}x{n}: complete solve")
    g = gpu_solve(A, b, c, trace_cap=50 * (m + n))
    ref = oracle.solve(A, b, c, max_iter=K)
    assert g.status == oracle.OPTIMAL
    assert np.array_equal(g.trace[:K], ref.trace)
    rp, rd, gap = lp_checks.residuals(A, b, c, g.x, g.y)
    assert rp <= 1e-9 and rd <= 1e-9 and gap <= 1e-9, (rp, rd, gap)
    assert lp_checks.complementary_slackness(A, b, c, g.x, g.y) <= 1e-9
    assert abs(float(c @ g.x) - g.obj) <= 1e-9 * abs(g.obj)
    # The condensed tableau and two pivots per sweep take the same pivots and
    # end with the same bits.
    for schedule in (lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED, lpdense.SCHED_GRID_CONDENSED_PAIRED):
        gc = gpu_solve(A, b, c, trace_cap=50 * (m + n), schedule=schedule)
        assert gc.status == g.status and gc.iterations == g.iterations
        assert np.array_equal(gc.trace, g.trace)
        assert np.array_equal(bits(gc.x), bits(g.x)) and np.array_equal(bits(gc.y), bits(g.y))
        assert bits([gc.obj])[0] == bits([g.obj])[0] and np.array_equal(gc.basis, g.basis)
