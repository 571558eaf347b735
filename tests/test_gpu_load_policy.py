"""The grid kernels sweep with non-temporal tableau loads above 288 MiB of
stored constraint rows and with plain (temporal) loads below; each kernel has
a compiled variant per load policy.  The small parity cases of the other
tests therefore take the temporal variants, and the full-size goldens at
8192 x 8192 and 8192 x 1024 the non-temporal ones.  This runs small and
ragged cases on every grid schedule in a child process with
LPD_TEMPORAL_MAX_MB=0 (read once per process), so that every kernel takes
its non-temporal variant, and compares them with the oracle bit for bit."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DONE = "non-temporal variants equal the oracle"

CHILD = r'''
import sys
import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import assert_bitwise_equal, gpu_solve
scheds = [lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED, lpdense.SCHED_GRID_PAIRED,
          lpdense.SCHED_GRID_CONDENSED_PAIRED]
for m, n, seed in [(64, 64, 3), (257, 130, 1), (700, 900, 4), (1025, 1023, 2)]:
    A, b, c = lpgen.dense_lp(m, n, seed)
    ref = oracle.solve(A, b, c, want_tableau=True)
    for s in scheds:
        print(f"[gpu-case] non-temporal loads {m}x{n} seed={seed} schedule={s}", file=sys.stderr, flush=True)
        g = gpu_solve(A, b, c, schedule=s, want_tableau=True)
        assert_bitwise_equal(g, ref, check_tableau=True)
print("%s", flush=True)
''' % DONE


def test_non_temporal_variants_in_a_child_process():
    env = dict(os.environ, LPD_TEMPORAL_MAX_MB="0")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=100)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert DONE in r.stdout
