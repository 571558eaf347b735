"""The grid kernels sweep with non-temporal tableau loads above 288 MiB of
stored constraint rows and with plain (temporal) loads below; each kernel has
a compiled variant per load policy.  The small parity cases of the other
tests therefore take the temporal variants, and the full-size goldens at
8192 x 8192 and 8192 x 1024 the non-temporal ones.  This runs small and
ragged cases on every grid schedule with LPD_TEMPORAL_MAX_MB=0 (the library
reads it at every launch), so that every kernel takes its non-temporal
variant, and compares them with the oracle bit for bit.  It runs in the
test process: a child process's first grid launch failed with a HIP runtime
error once this process had made cooperative launches of its own."""
import os

import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, assert_bitwise_equal, gpu_solve

pytestmark = pytest.mark.gpu

SCHEDULES = [lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED,
             lpdense.SCHED_GRID_CONDENSED_PAIRED]


@pytest.fixture
def non_temporal():
    old = os.environ.get("LPD_TEMPORAL_MAX_MB")
    os.environ["LPD_TEMPORAL_MAX_MB"] = "0"
    try:
        yield
    finally:
        if old is None:
            del os.environ["LPD_TEMPORAL_MAX_MB"]
        else:
            os.environ["LPD_TEMPORAL_MAX_MB"] = old


@pytest.mark.parametrize("m,n,seed", [(64, 64, 3), (257, 130, 1), (700, 900, 4), (1025, 1023, 2)])
def test_non_temporal_variants(m, n, seed, non_temporal):
    A, b, c = lpgen.dense_lp(m, n, seed)
    ref = oracle.solve(A, b, c, want_tableau=True)
    for s in SCHEDULES:
        announce(f"non-temporal loads {m}x{n} seed={seed} schedule={s}")
        g = gpu_solve(A, b, c, schedule=s, want_tableau=True)
        assert_bitwise_equal(g, ref, check_tableau=True)
