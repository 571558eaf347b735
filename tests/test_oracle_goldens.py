"""The stored whole-solve results (tests/golden/*.npz, written by
tests/golden/make_oracle_goldens.py from the CPU oracle alone) are the
oracle's as it stands: the cheap ones are recomputed here and must agree bit
for bit (CPU only; the 8192 x 8192 solve takes minutes and is not rerun)."""
import hashlib
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpgen
from tests import lp_checks

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("m,n", [(8192, 8192), (4096, 4096), (8192, 1024), (1024, 8192), (2048, 8192)])
def test_fullsize_golden_is_consistent(m, n):
    """Every stored solve is optimal, its trace has one (k, l) per pivot
    with k a column and l a row, the final basis is the trace's, and x, z
    read back from it agree (z = c^T x within 1e-9)."""
    g = _load(f"fullsize_{m}x{n}_seed0.npz")
    assert int(g["status"]) == oracle.OPTIMAL and g["trace"].shape == (int(g["iterations"]), 2)
    assert np.all((g["trace"][:, 0] >= 0) & (g["trace"][:, 0] < n + m))
    assert np.all((g["trace"][:, 1] >= 0) & (g["trace"][:, 1] < m))
    basis = np.arange(n, n + m)
    for k, l in g["trace"]:
        basis[l] = k
    assert np.array_equal(basis, g["basis"])
    x = g["x_bits"].view(np.float64)
    A, b, c = lpgen.dense_lp(m, n, 0)
    z = g["obj_bits"].view(np.float64)[0]
    assert abs(float(c @ x) - z) <= 1e-9 * abs(z)
    rp, rd, gap = lp_checks.residuals(A, b, c, x, g["y_bits"].view(np.float64))
    assert max(rp, rd, gap) <= 1e-9


def test_fullsize_golden_recomputed():
    """1024 x 8192 (409 pivots, seconds on one core) is rerun bit for bit."""
    g = _load("fullsize_1024x8192_seed0.npz")
    A, b, c = lpgen.dense_lp(1024, 8192, 0)
    r = oracle.solve(A, b, c)
    assert r.status == int(g["status"]) and r.iterations == int(g["iterations"])
    assert np.array_equal(r.trace, g["trace"])
    assert np.array_equal(r.basis, g["basis"].astype(np.int64))
    assert np.array_equal(r.x.view(np.int64), g["x_bits"]) and np.array_equal(r.y.view(np.int64), g["y_bits"])
    assert np.array([r.obj]).view(np.int64)[0] == g["obj_bits"][0]


def test_batch_golden_recomputed_sample():
    g = _load("batch1024_seed0.npz")
    assert int(g["count"]) == 1024 and np.all(g["status"] == oracle.OPTIMAL)
    for i in np.random.default_rng(3).choice(1024, 24, replace=False):
        A, b, c = lpgen.batch_lp(int(i), 1024, 32, 1024, 0)
        r = oracle.solve(A, b, c)
        assert r.iterations == int(g["iterations"][i]), i
        assert np.array([r.obj]).view(np.int64)[0] == g["obj_bits"][i], i
        assert hashlib.sha256(np.ascontiguousarray(r.x, dtype="<f8").tobytes()).digest() == g["x_sha256"][i].tobytes()
