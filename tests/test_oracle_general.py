"""Pins of the two-phase reference (oracle/general.py) against scipy's HiGHS
and against the paper-method oracle where no phase I is needed."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from oracle import general
from paper_1804_04737_amd import lpgen
from tests.gpu_util import bits


def _highs(A, b, c, sense):
    le, eq = sense == 0, sense == 1
    ge = sense == 2
    A_ub = np.vstack([A[le], -A[ge]])
    b_ub = np.concatenate([b[le], -b[ge]])
    r = linprog(-c, A_ub=A_ub if len(A_ub) else None, b_ub=b_ub if len(b_ub) else None,
                A_eq=A[eq] if eq.any() else None, b_eq=b[eq] if eq.any() else None,
                bounds=[(0, None)] * A.shape[1], method="highs")
    return r


@pytest.mark.parametrize("m,n,seed", [(3, 4, 0), (5, 5, 1), (8, 12, 2), (20, 15, 3), (40, 60, 4), (120, 90, 5)])
def test_general_matches_highs(m, n, seed):
    A, b, c, sense = lpgen.general_lp(m, n, seed)
    r = general.solve_general(A, b, c, sense)
    h = _highs(A, b, c, sense)
    assert h.status == 0 and r.status == oracle.OPTIMAL
    assert abs(r.obj - (-h.fun)) <= 1e-9 * max(1.0, abs(h.fun))
    x = r.x
    scale = 1.0 + np.abs(b).max()
    ax = A @ x
    assert np.all(x >= -1e-9)
    assert np.all(ax[sense == 0] <= b[sense == 0] + 1e-9 * scale)
    assert np.all(ax[sense == 2] >= b[sense == 2] - 1e-9 * scale)
    assert np.all(np.abs(ax[sense == 1] - b[sense == 1]) <= 1e-9 * scale)


def test_general_infeasible_and_unbounded():
    # x1 + x2 = -1 has no solution with x >= 0.
    A = np.array([[1.0, 1.0], [1.0, 0.0]])
    r = general.solve_general(A, np.array([-1.0, 5.0]), np.array([1.0, 1.0]), np.array([1, 0], np.int8))
    assert r.status == general.INFEASIBLE
    # x1 >= 1, x2 >= 2, maximise x1 + x2: unbounded after phase I.
    A = np.array([[1.0, 0.0], [0.0, 1.0]])
    r = general.solve_general(A, np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([2, 2], np.int8))
    assert r.status == oracle.UNBOUNDED


def test_general_degenerate_artificial_and_square_system():
    # Two identical equality rows: one artificial stays basic at level zero.
    A = np.array([[1.0, 2.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 1.0]])
    b = np.array([4.0, 4.0, 10.0])
    c = np.array([1.0, 1.0, 3.0])
    sense = np.array([1, 1, 0], np.int8)
    r = general.solve_general(A, b, c, sense)
    h = _highs(A, b, c, sense)
    assert r.status == oracle.OPTIMAL and abs(r.obj - (-h.fun)) <= 1e-9
    assert abs(A[0] @ r.x - 4.0) <= 1e-12
    # A square nonsingular equality system: phase II has no structural column.
    A = np.array([[2.0, 1.0], [1.0, 3.0]])
    r = general.solve_general(A, np.array([5.0, 10.0]), np.array([1.0, 1.0]), np.array([1, 1], np.int8))
    assert r.status == oracle.OPTIMAL
    assert np.allclose(r.x, [1.0, 3.0], atol=1e-12)


def test_general_reduces_to_the_paper_method_without_artificials():
    A, b, c = lpgen.dense_lp(30, 40, 9)
    r = general.solve_general(A, b, c)
    ref = oracle.solve(A, b, c)
    assert r.status == ref.status and r.iterations == ref.iterations
    assert np.array_equal(bits(r.x), bits(ref.x))
