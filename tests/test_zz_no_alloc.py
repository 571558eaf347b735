"""lp_solve_dense_noalloc (the entry point for callers that cannot allocate
device memory) gives bit for bit what lp_solve_dense_ex gives, on every
schedule, for two calls in a row that share the library's fixed workspace
(the second on a smaller LP), and rejects a workspace beyond its limit."""
import numpy as np
import pytest

from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu

SCHEDULES = [lpdense.SCHED_AUTO, lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED,
             lpdense.SCHED_GRID_CONDENSED_PAIRED]


def _dev(A, b, c):
    import torch
    d = torch.device("cuda:0")
    return tuple(torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(d) for v in (A, b, c))


def _host(r, m, n):
    import torch
    torch.cuda.synchronize()
    it = int(r.iterations.item())
    return dict(status=int(r.status.item()), it=it, x=bits(r.x.cpu().numpy()), obj=bits(r.obj.cpu().numpy()),
                y=bits(r.y.cpu().numpy()), basis=r.basis.cpu().numpy(), trace=r.trace.cpu().numpy()[:it])


@pytest.mark.parametrize("schedule", SCHEDULES, ids=["auto", "grid", "condensed", "paired", "condensed_paired"])
def test_noalloc_equals_ex_twice(schedule):
    # Second call smaller than the first: a stale first-call workspace (ticket
    # counters, barrier slots, tableau rows) must not leak into it.
    for (m, n, seed) in ((700, 900, 1), (130, 95, 2)):
        A, b, c = lpgen.dense_lp(m, n, seed)
        tA, tb, tc = _dev(A, b, c)
        announce(f"noalloc {m}x{n} seed={seed} schedule={schedule}")
        kw = dict(schedule=schedule, trace_cap=50 * (m + n), want_basis=True)
        ref = _host(lpdense.solve_dense_ex(tA, tb, tc, **kw), m, n)
        got = _host(lpdense.solve_dense_ex(tA, tb, tc, noalloc=True, **kw), m, n)
        assert got["status"] == ref["status"] == lpdense.OPTIMAL and got["it"] == ref["it"]
        assert np.array_equal(got["trace"], ref["trace"])
        for key in ("x", "obj", "y", "basis"):
            assert np.array_equal(got[key], ref[key]), key


def test_noalloc_iteration_cap_and_stale_state():
    # An iteration-limited call, then a full solve of another LP: the second
    # result is exactly lp_solve_dense_ex's.
    A1, b1, c1 = lpgen.dense_lp(900, 1200, 7)
    A2, b2, c2 = lpgen.dense_lp(400, 300, 8)
    t1, t2 = _dev(A1, b1, c1), _dev(A2, b2, c2)
    announce("noalloc capped call then a smaller full solve")
    r1 = lpdense.solve_dense_ex(*t1, schedule=lpdense.SCHED_GRID, max_iter=7, noalloc=True, want_basis=True,
                                trace_cap=7)
    e1 = lpdense.solve_dense_ex(*t1, schedule=lpdense.SCHED_GRID, max_iter=7, want_basis=True, trace_cap=7)
    g1, f1 = _host(r1, 900, 1200), _host(e1, 900, 1200)
    assert g1["status"] == f1["status"] == lpdense.ITERATION_LIMIT
    assert all(np.array_equal(g1[k], f1[k]) for k in ("x", "obj", "y", "basis", "trace"))
    r2 = lpdense.solve_dense_ex(*t2, schedule=lpdense.SCHED_GRID_CONDENSED, noalloc=True, want_basis=True,
                                trace_cap=4000)
    e2 = lpdense.solve_dense_ex(*t2, schedule=lpdense.SCHED_GRID_CONDENSED, want_basis=True, trace_cap=4000)
    g2, f2 = _host(r2, 400, 300), _host(e2, 400, 300)
    assert g2["status"] == f2["status"] == lpdense.OPTIMAL
    assert all(np.array_equal(g2[k], f2[k]) for k in ("x", "obj", "y", "basis", "trace"))


def test_noalloc_rejects_workspace_beyond_its_limit():
    # 3000 x 3000 on the full tableau needs ~140 MiB of workspace (limit 128 MiB):
    # rejected on the host, nothing enqueued; the condensed tableau fits.
    A, b, c = lpgen.dense_lp(3000, 3000, 3)
    tA, tb, tc = _dev(A, b, c)
    announce("noalloc size limit")
    with pytest.raises(lpdense.LpdError) as ei:
        lpdense.solve_dense_ex(tA, tb, tc, schedule=lpdense.SCHED_GRID, noalloc=True)
    assert ei.value.code == -7  # LPD_ERR_TOO_LARGE
    r = lpdense.solve_dense_ex(tA, tb, tc, schedule=lpdense.SCHED_GRID_CONDENSED, max_iter=5, noalloc=True)
    e = lpdense.solve_dense_ex(tA, tb, tc, schedule=lpdense.SCHED_GRID_CONDENSED, max_iter=5)
    g, f = _host_small(r), _host_small(e)
    assert g == f


def _host_small(r):
    import torch
    torch.cuda.synchronize()
    return (int(r.status.item()), int(r.iterations.item()), r.x.cpu().numpy().tobytes(), r.obj.cpu().numpy().tobytes())
