"""Input generators: determinism and the stated distributions (they hold no
simplex arithmetic, so these are the only checks they need)."""
import numpy as np

import oracle
from paper_1804_04737_amd import lpgen
from tests import lp_checks


def test_dense_lp_distribution_and_determinism():
    A, b, c = lpgen.dense_lp(50, 70, 3)
    A2, b2, c2 = lpgen.dense_lp(50, 70, 3)
    assert np.array_equal(A, A2) and np.array_equal(b, b2) and np.array_equal(c, c2)
    assert A.min() >= 1 and A.max() <= 100 and np.all(A == np.round(A))
    s = 70 / 64.0
    assert b.min() >= 1000 * s and b.max() <= 10000 * s
    assert c.min() >= 1 and c.max() <= 100


def test_paper_lp_distribution_and_determinism():
    A, b, c = lpgen.paper_lp(300, 200, 7)
    A2, b2, c2 = lpgen.paper_lp(300, 200, 7)
    assert np.array_equal(A, A2) and np.array_equal(b, b2) and np.array_equal(c, c2)
    nz = A != 0
    assert abs(nz.mean() - 0.9) < 0.01
    assert A.min() >= 0 and A.max() <= 50 and np.all(A == np.round(A)) and A[nz].min() >= 1
    assert np.all(b >= 0) and np.all(b == np.round(b))
    assert np.any(c > 0) and np.any(c < 0)
    assert np.all(nz.any(axis=0))  # no empty column: the LP is bounded


def test_paper_lp_solves_to_optimality_with_certificates():
    """Small paper-style instances reach OPTIMAL in the oracle with zero
    duality gap, and match brute-force vertex enumeration on tiny ones."""
    for seed in range(6):
        A, b, c = lpgen.paper_lp(4, 5, seed)
        r = oracle.solve(A, b, c)
        assert r.status == oracle.OPTIMAL
        best, _ = lp_checks.brute_force_optimum(A, b, c)
        assert abs(r.obj - best) <= 1e-9 * max(1.0, abs(best))
    for seed in range(3):
        A, b, c = lpgen.paper_lp(60, 80, 100 + seed)
        r = oracle.solve(A, b, c)
        assert r.status == oracle.OPTIMAL
        rp, rd, gap = lp_checks.residuals(A, b, c, r.x, r.y)
        assert rp <= 1e-9 and rd <= 1e-9 and gap <= 1e-9
