"""lp_solve_tableau (Steps 2-5 from a given basic tableau) equals the oracle's
oracle.solve_tableau bit for bit on every schedule: pivot sequence, final
tableau, basis, x and z.  Starts: Table 1 itself, the tableau after K oracle
pivots (the continuation must be the rest of the full solve), and the
phase I tableau of a general LP (artificial basis, objective row priced)."""
import numpy as np
import pytest

import oracle
from oracle import general
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu

SCHEDULES = [(lpdense.SCHED_AUTO, "auto"), (lpdense.SCHED_GRID, "grid"), (lpdense.SCHED_GRID_CONDENSED, "condensed"),
             (lpdense.SCHED_GRID_PAIRED, "paired"), (lpdense.SCHED_GRID_CONDENSED_PAIRED, "condensed_paired")]


def _gpu(T0, basis0, schedule, max_iter=-1):
    import torch
    m, ncols = T0.shape[0] - 1, T0.shape[1] - 1
    cap = 50 * ncols if max_iter < 0 else max(max_iter, 1)
    r = lpdense.solve_tableau(torch.from_numpy(np.ascontiguousarray(T0)).to("cuda:0"), basis0, schedule=schedule,
                              max_iter=max_iter, trace_cap=cap, want_basis=True, want_tableau=True)
    torch.cuda.synchronize()
    it = int(r.iterations.item())
    return dict(status=int(r.status.item()), it=it, trace=r.trace.cpu().numpy()[:min(it, cap)],
                basis=r.basis.cpu().numpy(), tableau=r.tableau.cpu().numpy(), x=r.x.cpu().numpy(),
                obj=float(r.obj.item()))


def _check(T0, basis0, max_iter=None, schedules=SCHEDULES):
    ref = oracle.solve_tableau(T0, basis0, max_iter=max_iter)
    for sched, name in schedules:
        g = _gpu(T0, basis0, sched, -1 if max_iter is None else max_iter)
        assert g["status"] == ref.status and g["it"] == ref.iterations, (name, g["status"], ref.status)
        if not np.array_equal(g["trace"], ref.trace):
            bad = int(np.argmax(np.any(g["trace"] != ref.trace, axis=1)))
            raise AssertionError(f"{name}: pivot {bad}: gpu {g['trace'][bad]} oracle {ref.trace[bad]}")
        assert np.array_equal(g["basis"], ref.basis), name
        same = bits(g["tableau"]) == bits(ref.tableau)
        if not same.all():
            i, j = np.argwhere(~same)[0]
            raise AssertionError(f"{name}: tableau differs first at ({i},{j})")
        assert np.array_equal(bits(g["x"]), bits(ref.x)), name
        assert bits([g["obj"]])[0] == bits([ref.obj])[0], name
    return ref


def _table1(A, b, c):
    m, n = A.shape
    T = np.zeros((m + 1, n + m + 1))
    T[:m, :n] = A
    T[:m, n:n + m] = np.eye(m)
    T[:m, -1] = b
    T[m, :n] = -c
    return T, np.arange(n, n + m)


@pytest.mark.parametrize("m,n,seed", [(20, 30, 1), (64, 64, 0), (300, 400, 2), (700, 500, 3)])
def test_table1_start_equals_dense_solve(m, n, seed):
    """From Table 1 with the slack basis the tableau start is the paper's
    solve: same pivots and bits as oracle.solve."""
    A, b, c = lpgen.dense_lp(m, n, seed)
    T, basis = _table1(A, b, c)
    announce(f"tableau start from Table 1 {m}x{n} seed={seed}")
    ref = _check(T, basis)
    full = oracle.solve(A, b, c)
    assert np.array_equal(ref.trace, full.trace) and ref.status == full.status


@pytest.mark.parametrize("m,n,seed,K", [(40, 60, 4, 3), (300, 200, 5, 25), (500, 900, 6, 60)])
def test_continuation_after_k_pivots(m, n, seed, K):
    """Start from the oracle's tableau after K pivots: the GPU continuation
    equals the oracle's continuation, which is the rest of the full solve."""
    A, b, c = lpgen.dense_lp(m, n, seed)
    mid = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    assert mid.status == oracle.ITERATION_LIMIT
    announce(f"tableau start after {K} pivots {m}x{n} seed={seed}")
    ref = _check(mid.tableau, mid.basis)
    full = oracle.solve(A, b, c)
    assert np.array_equal(ref.trace, full.trace[K:]) and ref.iterations == full.iterations - K


@pytest.mark.parametrize("m,n,seed", [(8, 12, 2), (60, 80, 11), (300, 400, 6)])
def test_phase1_tableau_start(m, n, seed):
    """The phase I tableau of a general LP: artificial columns basic,
    objective row already priced."""
    A, b, c, sense = lpgen.general_lp(m, n, seed)
    T1, basis1 = general.phase1_tableau(A, b, sense)[:2]
    announce(f"phase I tableau start {m}x{n} seed={seed}")
    _check(T1, basis1)


def test_wide_rows_and_edge_cases():
    # A pivot row longer than the LDS holds (column panels on the grid).
    A, b, c = lpgen.dense_lp(24, 20000, 7)
    mid = oracle.solve(A, b, c, max_iter=3, want_tableau=True)
    announce("tableau start with rows longer than the LDS")
    _check(mid.tableau, mid.basis, schedules=SCHEDULES[1:])
    # Every column basic: optimal at once.
    T = np.zeros((4, 4))
    T[:3, :3] = np.eye(3)
    T[:3, 3] = [1.0, 2.0, 3.0]
    T[3, 3] = 6.0
    _check(T, np.arange(3))
    # Iteration caps 0 and 1.
    A, b, c = lpgen.dense_lp(50, 70, 8)
    T, basis = _table1(A, b, c)
    _check(T, basis, max_iter=0)
    _check(T, basis, max_iter=1)
    # A NaN anywhere in the tableau: NUMERICAL before any pivot.
    T[10, 30] = np.nan
    ref = _check(T, basis)
    assert ref.status == oracle.NUMERICAL and ref.iterations == 0


def test_invalid_basis_rejected_on_host():
    import torch
    T = torch.zeros((3, 5), dtype=torch.float64, device="cuda:0")
    for bad in ([0, 0], [0, 4], [-1, 1]):
        with pytest.raises(lpdense.LpdError) as ei:
            lpdense.solve_tableau(T, bad)
        assert ei.value.code == -1
