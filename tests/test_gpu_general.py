"""General LPs (lp_solve_general, two-phase method) reproduce the two-phase
reference bit for bit: status, pivots of both phases, x and c^T x."""
import numpy as np
import pytest

from oracle import general
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu


def _gpu(A, b, c, sense, schedule=lpdense.SCHED_AUTO, max_iter=-1):
    import torch
    dev = torch.device("cuda")
    tA, tb, tc = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(dev) for v in (A, b, c))
    r = lpdense.solve_general(tA, tb, tc, sense, schedule=schedule, max_iter=max_iter)
    return int(r.status.item()), r.x.cpu().numpy(), float(r.obj.item()), int(r.iterations.item())


def _check(A, b, c, sense, schedule=lpdense.SCHED_AUTO, max_iter=-1):
    st, x, obj, it = _gpu(A, b, c, sense, schedule, max_iter)
    ref = general.solve_general(A, b, c, sense, max_iter=None if max_iter < 0 else max_iter)
    assert st == ref.status and it == ref.iterations, (st, ref.status, it, ref.iterations)
    assert np.array_equal(bits(x), bits(ref.x))
    assert bits([obj])[0] == bits([ref.obj])[0]
    return st


@pytest.mark.parametrize("schedule", [lpdense.SCHED_AUTO, lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED,
                                      lpdense.SCHED_GRID_PAIRED, lpdense.SCHED_GRID_CONDENSED_PAIRED],
                         ids=["auto", "grid", "condensed", "paired", "condensed_paired"])
@pytest.mark.parametrize("m,n,seed", [(3, 4, 0), (20, 15, 3), (120, 90, 5), (300, 400, 6), (700, 500, 7)])
def test_general_equals_reference(m, n, seed, schedule):
    A, b, c, sense = lpgen.general_lp(m, n, seed)
    announce(f"general {m}x{n} seed={seed} schedule={schedule}")
    assert _check(A, b, c, sense, schedule) == lpdense.OPTIMAL


def test_general_edge_cases():
    announce("general edge cases")
    A = np.array([[1.0, 1.0], [1.0, 0.0]])
    assert _check(A, np.array([-1.0, 5.0]), np.array([1.0, 1.0]), np.array([1, 0], np.int8)) == lpdense.INFEASIBLE
    A = np.eye(2)
    assert _check(A, np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([2, 2], np.int8)) == lpdense.UNBOUNDED
    A = np.array([[1.0, 2.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 1.0]])
    assert _check(A, np.array([4.0, 4.0, 10.0]), np.array([1.0, 1.0, 3.0]),
                  np.array([1, 1, 0], np.int8)) == lpdense.OPTIMAL
    A = np.array([[2.0, 1.0], [1.0, 3.0]])
    assert _check(A, np.array([5.0, 10.0]), np.array([1.0, 1.0]), np.array([1, 1], np.int8)) == lpdense.OPTIMAL
    # Only <= rows with b >= 0: one solve, same pivots as the paper-method path.
    A, b, c = lpgen.dense_lp(50, 60, 2)
    assert _check(A, b, c, None) == lpdense.OPTIMAL
    # >= rows with b <= 0 need no artificial either.
    A, b, c = lpgen.dense_lp(40, 30, 4)
    assert _check(-A, -b, c, np.full(40, 2, np.int8)) == lpdense.OPTIMAL
    # NaN in A: phase I reports NUMERICAL.
    A, b, c, sense = lpgen.general_lp(10, 10, 1)
    A[3, 4] = np.nan
    assert _check(A, b, c, sense) == lpdense.NUMERICAL
    # Iteration cap in phase II.
    A, b, c, sense = lpgen.general_lp(60, 80, 11)
    _check(A, b, c, sense, max_iter=3)
