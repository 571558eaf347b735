"""The bounded barrier waits of the grid schedules end a solve with
LPD_DEVICE_TIMEOUT instead of hanging.  With the watchdog option set to "no
wait at all" every wait of a multi-workgroup team gives up at once, so every
workgroup leaves the persistent kernel normally with that status; the device
stays healthy and the next solve on the same stream gives the oracle's bits.
(The condition is forced from the host: no kernel faults or hangs.)"""
import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu

SCHEDULES = [(lpdense.SCHED_GRID, "grid"), (lpdense.SCHED_GRID_CONDENSED, "condensed"),
             (lpdense.SCHED_GRID_PAIRED, "paired"), (lpdense.SCHED_GRID_CONDENSED_PAIRED, "condensed_paired")]


@pytest.mark.parametrize("schedule,name", SCHEDULES, ids=[s[1] for s in SCHEDULES])
@pytest.mark.parametrize("grid_blocks", [0, 4])
def test_every_wait_gives_up(schedule, name, grid_blocks):
    import torch
    A, b, c = lpgen.dense_lp(300, 400, 3)
    dev = torch.device("cuda:0")
    tA, tb, tc = (torch.from_numpy(v).to(dev) for v in (A, b, c))
    announce(f"watchdog: no wait, {name}, grid_blocks={grid_blocks}")
    r = lpdense.solve_dense_ex(tA, tb, tc, schedule=schedule, grid_blocks=grid_blocks, watchdog_us=-1)
    torch.cuda.synchronize()
    assert int(r.status.item()) == lpdense.DEVICE_TIMEOUT
    # A generous explicit bound and then the default: normal solves, exact.
    ref = oracle.solve(A, b, c)
    for wd in (5_000_000, 0):
        g = lpdense.solve_dense_ex(tA, tb, tc, schedule=schedule, grid_blocks=grid_blocks, watchdog_us=wd)
        torch.cuda.synchronize()
        assert int(g.status.item()) == ref.status and int(g.iterations.item()) == ref.iterations
        assert np.array_equal(bits(g.x.cpu().numpy()), bits(ref.x))
        assert bits([float(g.obj.item())])[0] == bits([ref.obj])[0]
