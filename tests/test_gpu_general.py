"""General LPs (lp_solve_general, the two-phase method) equal the textbook
two-phase reference oracle/general.py bit for bit on every schedule:
status, pivots of both phases and the drive-out, x and z.  The reference is
pinned on its own by tests/test_oracle_general.py (brute force, a basis
certificate, hand-derived pivot sequences, HiGHS)."""
import json
import os

import numpy as np
import pytest

from oracle import general
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits
from tests.test_oracle_general import _tiny_cases

pytestmark = pytest.mark.gpu

SCHEDULES = [lpdense.SCHED_AUTO, lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED,
             lpdense.SCHED_GRID_CONDENSED_PAIRED]
IDS = ["auto", "grid", "condensed", "paired", "condensed_paired"]
EXAMPLES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "general_examples.json")


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
    return st, ref


@pytest.mark.parametrize("schedule", SCHEDULES, ids=IDS)
@pytest.mark.parametrize("m,n,seed", [(3, 4, 0), (20, 15, 3), (120, 90, 5), (300, 400, 6), (700, 500, 7)])
def test_general_equals_reference(m, n, seed, schedule):
    A, b, c, sense = lpgen.general_lp(m, n, seed)
    announce(f"general {m}x{n} seed={seed} schedule={schedule}")
    assert _check(A, b, c, sense, schedule)[0] == lpdense.OPTIMAL


@pytest.mark.parametrize("schedule", SCHEDULES, ids=IDS)
def test_general_hand_examples_and_tiny_lps(schedule):
    """The hand-derived examples (drive-out pivot, redundant row, negative
    right-hand side) and 90 tiny LPs of every status, with drive-out pivots
    and redundant rows among them."""
    announce(f"general hand examples and tiny LPs schedule={schedule}")
    with open(EXAMPLES) as f:
        for ex in json.load(f)["examples"]:
            st, _ = _check(np.array(ex["A"], float), np.array(ex["b"], float), np.array(ex["c"], float),
                           np.array(ex["sense"], np.int8), schedule)
            assert st == ex["status"]
    drive = redundant = 0
    seen = set()
    for A, b, c, sense in _tiny_cases(60):
        st, ref = _check(A, b, c, sense, schedule)
        seen.add(st)
        drive += ref.driveout_pivots
        redundant += ref.rows is not None and len(ref.rows) < A.shape[0]
    assert {lpdense.OPTIMAL, lpdense.UNBOUNDED, lpdense.INFEASIBLE} <= seen and drive and redundant


def test_general_edge_cases():
    announce("general edge cases")
    A = np.array([[1.0, 1.0], [1.0, 0.0]])
    assert _check(A, np.array([-1.0, 5.0]), np.array([1.0, 1.0]), np.array([1, 0], np.int8))[0] == lpdense.INFEASIBLE
    assert _check(np.eye(2), np.array([1.0, 2.0]), np.array([1.0, 1.0]),
                  np.array([2, 2], np.int8))[0] == lpdense.UNBOUNDED
    A = np.array([[1.0, 2.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 1.0]])
    assert _check(A, np.array([4.0, 4.0, 10.0]), np.array([1.0, 1.0, 3.0]),
                  np.array([1, 1, 0], np.int8))[0] == lpdense.OPTIMAL
    A = np.array([[2.0, 1.0], [1.0, 3.0]])
    assert _check(A, np.array([5.0, 10.0]), np.array([1.0, 1.0]), np.array([1, 1], np.int8))[0] == lpdense.OPTIMAL
    # Every row redundant: phase II has no constraint row.
    for cc, want in ((np.array([1.0, -1.0]), lpdense.UNBOUNDED), (np.array([-1.0, -2.0]), lpdense.OPTIMAL)):
        assert _check(np.zeros((2, 2)), np.zeros(2), cc, np.array([1, 1], np.int8))[0] == want
    # Only <= rows with b >= 0: phase I ends at once, phase II is Table 1.
    A, b, c = lpgen.dense_lp(50, 60, 2)
    assert _check(A, b, c, None)[0] == lpdense.OPTIMAL
    # >= rows with b <= 0 need no artificial either.
    A, b, c = lpgen.dense_lp(40, 30, 4)
    assert _check(-A, -b, c, np.full(40, 2, np.int8))[0] == lpdense.OPTIMAL
    # NaN in A: phase I reports NUMERICAL.
    A, b, c, sense = lpgen.general_lp(10, 10, 1)
    A[3, 4] = np.nan
    assert _check(A, b, c, sense)[0] == lpdense.NUMERICAL
    # Iteration caps in phase I and in phase II.
    A, b, c, sense = lpgen.general_lp(60, 80, 11)
    for cap in (0, 3, 40):
        _check(A, b, c, sense, max_iter=cap)
