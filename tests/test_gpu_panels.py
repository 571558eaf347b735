"""Pivot rows longer than the LDS holds.

The grid schedules keep the normalised pivot row in LDS.  A row of more
vectors (16 bytes each) than fit next to the capture list is swept in column
panels: every workgroup forms the panel of the normalised row it needs from
the pivot row itself, with the same division as the pricing phase, so the
bits are those of the oracle.  Cases: 2 to 5 panels, the static chunk order
(whole grid, short sweep) and the ticket-driven one (small grids, long
sweeps), both tableau forms, a many-row LP whose sweep is long on the whole
grid, and the first pivots of a 32768 x 32768 LP, whose full tableau has more
than 2^31 elements.
"""
import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, assert_bitwise_equal, bits, gpu_solve

pytestmark = pytest.mark.gpu

GRID, CD, PAIR = lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED
CDPAIR = lpdense.SCHED_GRID_CONDENSED_PAIRED
LDS_BYTES = 160 * 1024
# Widest row that fits with a full capture list (scratch + 1024 entries of 20 B).
ROW_VECS_MAX = (LDS_BYTES - 32 * 24 - 16 - 1024 * 20) // 16


def stored_vecs(m, n, schedule):
    return (n + 1) // 2 if schedule in (CD, CDPAIR) else (n + m + 1) // 2


@pytest.mark.parametrize("m,n,blocks,schedule", [
    (64, 20000, 0, GRID), (64, 20000, 2, GRID), (64, 20000, 7, GRID),
    (40, 45000, 0, GRID), (40, 45000, 3, GRID), (24, 80000, 2, GRID),
    (64, 20000, 0, CD), (64, 20000, 2, CD), (40, 45000, 3, CD),
    (64, 20000, 0, PAIR), (64, 20000, 2, PAIR), (24, 80000, 2, PAIR),
    (64, 20000, 0, CDPAIR), (40, 45000, 3, CDPAIR), (24, 80000, 2, CDPAIR),
], ids=lambda v: str(v))
def test_panelled_rows_bitwise(m, n, blocks, schedule):
    assert stored_vecs(m, n, schedule) > ROW_VECS_MAX  # the panelled kernel runs
    A, b, c = lpgen.dense_lp(m, n, 3)
    announce(f"panels {m}x{n} blocks={blocks} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, grid_blocks=blocks, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert ref.status == oracle.OPTIMAL
    assert_bitwise_equal(g, ref, check_tableau=True)


@pytest.mark.parametrize("schedule", [GRID, CD], ids=["grid", "condensed"])
def test_panelled_many_rows(schedule):
    """2048 x 30000: two panels and a ticket-driven sweep on the whole grid.
    The first 8 pivots against the oracle's tableau (sampled rows, the whole
    objective row and right-hand side)."""
    m, n, K = 2048, 30000, 8
    assert stored_vecs(m, n, schedule) > ROW_VECS_MAX
    A, b, c = lpgen.dense_lp(m, n, 4)
    announce(f"panels {m}x{n} first {K} pivots schedule={schedule}")
    ref = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    g = gpu_solve(A, b, c, schedule=schedule, max_iter=K, want_tableau=True)
    assert g.status == ref.status == oracle.ITERATION_LIMIT
    assert np.array_equal(g.trace, ref.trace)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, m, 48), ref.trace[:, 1], [m]]))
    assert np.array_equal(bits(g.tableau[rows]), bits(ref.tableau[rows]))
    assert np.array_equal(bits(g.tableau[:, -1]), bits(ref.tableau[:, -1]))
    assert np.array_equal(bits(g.x), bits(ref.x)) and np.array_equal(bits(g.y), bits(ref.y))


def test_more_than_2g_tableau_elements():
    """32768 x 32768: the full tableau is 32769 x 65537 = 2,147,581,953
    doubles (17.2 GB), past 2^31 elements, in four panels; the condensed one
    (1.07e9 doubles) in two.  The first 2 pivots against the oracle."""
    m = n = 32768
    K = 2
    A, b, c = lpgen.dense_lp(m, n, 0)
    announce(f"max size {m}x{n}: oracle, first {K} pivots")
    ref = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([rng.integers(0, m, 24), ref.trace[:, 1], [m]]))
    ref_rows = ref.tableau[rows].copy()
    ref_rhs = ref.tableau[:, -1].copy()
    ref.tableau = None
    for schedule in (GRID, CD):
        announce(f"max size {m}x{n}: first {K} pivots schedule={schedule}")
        g = gpu_solve(A, b, c, schedule=schedule, max_iter=K, want_tableau=True)
        assert g.status == ref.status == oracle.ITERATION_LIMIT
        assert np.array_equal(g.trace, ref.trace)
        assert np.array_equal(bits(g.tableau[rows]), bits(ref_rows))
        assert np.array_equal(bits(g.tableau[:, -1]), bits(ref_rhs))
        assert np.array_equal(bits(g.x), bits(ref.x)) and np.array_equal(bits(g.y), bits(ref.y))
        del g
