"""Pins of the CPU oracle to things other than itself (CPU only).

Each test checks the oracle against what the paper (Section 2, Steps 1-5;
Table 1) and LP theory fix: the initial-tableau layout, hand-derived worked
examples, brute-force vertex enumeration, closed forms, an LP library
(HiGHS), strong duality / complementary slackness, and the textbook
identities between a simplex tableau and its basis.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpgen
from tests import lp_checks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _examples():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["id"])
def test_worked_examples(ex):
    r = oracle.solve(np.array(ex["A"], float), np.array(ex["b"], float),
                     np.array(ex["c"], float), max_iter=ex.get("max_iter"))
    assert r.status == ex["status"]
    assert r.trace.tolist() == ex["trace"]
    np.testing.assert_allclose(r.x, ex["x"], rtol=0, atol=1e-12)
    assert abs(r.obj - ex["obj"]) <= 1e-12 * max(1, abs(ex["obj"]))
    np.testing.assert_allclose(r.y, ex["y"], rtol=0, atol=1e-12)


def test_initial_tableau_is_table1():
    """Step 1 / Table 1: [[A, I, b], [-c, 0, 0]] exactly (no pivot allowed)."""
    A, b, c = lpgen.dense_lp(7, 5, 3)
    r = oracle.solve(A, b, c, max_iter=0, want_tableau=True)
    assert r.status == oracle.ITERATION_LIMIT and r.iterations == 0
    want = np.block([[A, np.eye(7), b[:, None]], [-c[None, :], np.zeros((1, 7)), np.zeros((1, 1))]])
    assert np.array_equal(r.tableau, want)
    assert np.array_equal(r.basis, np.arange(5, 12))


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_vertices(seed):
    """Optimum equals the best basic feasible solution of [A | I] (m, n <= 5)."""
    rng = np.random.default_rng(1000 + seed)
    m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
    if seed % 2:
        A = rng.integers(1, 10, (m, n)).astype(float)      # integer data, many ties
        b = rng.integers(0, 20, m).astype(float)           # zeros -> degenerate
        c = rng.integers(-3, 10, n).astype(float)
    else:
        A = rng.uniform(0.1, 5.0, (m, n))
        b = rng.uniform(0.0, 10.0, m)
        c = rng.uniform(-1.0, 5.0, n)
    r = oracle.solve(A, b, c)
    assert r.status == oracle.OPTIMAL
    z, _ = lp_checks.brute_force_optimum(A, b, c)
    assert abs(r.obj - z) <= 1e-9 * max(1.0, abs(z))
    assert abs(float(c @ r.x) - r.obj) <= 1e-9 * max(1.0, abs(z))
    rp, rd, gap = lp_checks.residuals(A, b, c, r.x, r.y)
    assert rp <= 1e-12 and rd <= 1e-12 and gap <= 1e-12


@pytest.mark.parametrize("m,n,seed", [(64, 64, s) for s in range(5)] +
                         [(37, 91, 1), (120, 40, 2), (200, 200, 3), (300, 150, 4), (150, 300, 5)])
def test_highs_and_duality(m, n, seed):
    """Generator instances: optimum matches HiGHS; final tableau gives a
    feasible primal/dual pair with zero gap and complementary slackness."""
    A, b, c = lpgen.dense_lp(m, n, seed)
    r = oracle.solve(A, b, c)
    assert r.status == oracle.OPTIMAL
    z = lp_checks.highs_optimum(A, b, c)
    assert abs(r.obj - z) <= 1e-9 * max(1.0, abs(z))
    rp, rd, gap = lp_checks.residuals(A, b, c, r.x, r.y)
    assert rp <= 1e-9 and rd <= 1e-9 and gap <= 1e-9
    assert lp_checks.complementary_slackness(A, b, c, r.x, r.y) <= 1e-9


@pytest.mark.parametrize("m,n,seed,K", [(30, 20, 0, 5), (64, 64, 1, 9), (100, 150, 2, 15), (300, 300, 4, 40)])
def test_tableau_matches_basis_inverse(m, n, seed, K):
    """After K pivots the tableau equals B^-1 [A I b] with objective row
    c_B B^-1 [A I b] - [c 0 0] (Steps 4-5 applied K times), and the basic
    columns are exact unit vectors (fma(-f, 1, f) = 0 in IEEE arithmetic)."""
    A, b, c = lpgen.dense_lp(m, n, seed)
    full = oracle.solve(A, b, c)
    assert full.iterations >= 4
    K = min(K, full.iterations - 1)
    r = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    assert r.status == oracle.ITERATION_LIMIT and r.iterations == K
    assert np.array_equal(r.trace, full.trace[:K])
    errs = lp_checks.tableau_identity_errors(A, b, c, r.basis, r.tableau)
    assert max(errs.values()) <= 1e-9, errs
    T = r.tableau
    for i, j in enumerate(r.basis):
        col = T[:, j]
        unit = np.zeros(m + 1)
        unit[i] = 1.0
        assert np.array_equal(col, unit)


@pytest.mark.parametrize("n,seed", [(3, 0), (50, 1), (400, 2)])
def test_closed_form_diagonal(n, seed):
    """A = diag(d): column j only meets row j, so the entering order is the
    columns sorted by (-c_j, j), each leaving its own row; x_j = b_j / d_j."""
    rng = np.random.default_rng(seed)
    d = rng.integers(1, 9, n).astype(float)
    b = rng.integers(1, 50, n).astype(float)
    c = rng.integers(1, 6, n).astype(float)     # many equal costs -> ties
    r = oracle.solve(np.diag(d), b, c)
    order = sorted(range(n), key=lambda j: (-c[j], j))
    assert r.status == oracle.OPTIMAL
    assert r.trace.tolist() == [[j, j] for j in order]
    assert np.array_equal(r.x, b / d)
    z = float(np.sum(c * b / d))
    assert abs(r.obj - z) <= 1e-12 * z
    np.testing.assert_allclose(r.y, c / d, rtol=1e-15)


@pytest.mark.parametrize("m,seed", [(1, 0), (5, 1), (300, 2)])
def test_closed_form_single_variable(m, seed):
    """n = 1: one pivot; the leaving row is the lowest-index minimiser of
    b_i / a_i over a_i > 0, and z = c * min ratio."""
    rng = np.random.default_rng(seed)
    a = rng.integers(-2, 6, m).astype(float)
    a[rng.integers(0, m)] = 3.0
    b = rng.integers(0, 30, m).astype(float)
    c = np.array([2.5])
    r = oracle.solve(a[:, None], b, c)
    rho = np.where(a > 0, b / np.where(a > 0, a, 1), np.inf)
    l = int(np.argmin(rho))
    assert r.status == oracle.OPTIMAL
    assert r.trace.tolist() == [[0, l]]
    assert r.x[0] == b[l] / a[l]
    assert r.obj == 2.5 * (b[l] / a[l]) or abs(r.obj - 2.5 * b[l] / a[l]) <= 1e-15 * r.obj


@pytest.mark.parametrize("n,seed", [(1, 0), (8, 1), (500, 2)])
def test_closed_form_single_constraint(n, seed):
    """m = 1: z* = b * max_j c_j / a_j (a_j > 0)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 5.0, n)
    c = rng.uniform(0.5, 5.0, n)
    b = np.array([7.0])
    r = oracle.solve(a[None, :], b, c)
    assert r.status == oracle.OPTIMAL
    z = 7.0 * float(np.max(c / a))
    assert abs(r.obj - z) <= 1e-12 * z


def test_unbounded_column():
    """A column with no positive entry and a negative reduced cost: Step 3
    finds no ratio and the LP is unbounded."""
    A = np.array([[1.0, -1.0], [2.0, 0.0]])
    r = oracle.solve(A, np.array([4.0, 6.0]), np.array([1.0, 5.0]))
    assert r.status == oracle.UNBOUNDED and r.iterations == 0
    # After one pivot the unboundedness appears in a slack-generated column.
    A = np.array([[1.0, -1.0]])
    r = oracle.solve(A, np.array([1.0]), np.array([2.0, 1.0]))
    assert r.status == oracle.UNBOUNDED and r.trace.tolist() == [[0, 0]]


def test_preconditions():
    A = np.ones((2, 2))
    r = oracle.solve(A, np.array([1.0, -1.0]), np.ones(2))
    assert r.status == oracle.INFEASIBLE_START and r.iterations == 0
    assert r.obj == 0.0 and np.all(r.x == 0)
    A2 = A.copy()
    A2[1, 0] = np.nan
    assert oracle.solve(A2, np.ones(2), np.ones(2)).status == oracle.NUMERICAL
    assert oracle.solve(A, np.array([1.0, np.inf]), np.ones(2)).status == oracle.NUMERICAL
    # non-finite wins over a negative b
    assert oracle.solve(A2, np.array([1.0, -1.0]), np.ones(2)).status == oracle.NUMERICAL
    with pytest.raises(ValueError):
        oracle.solve(np.ones((0, 2)), np.ones(0), np.ones(2))


def test_iteration_cap_and_monotone_objective():
    """Capped runs reproduce the prefix of the full trace, and the objective
    never decreases from one pivot to the next (b >= 0 kept by the ratio test)."""
    A, b, c = lpgen.dense_lp(40, 60, 11)
    full = oracle.solve(A, b, c)
    prev = -np.inf
    for K in range(full.iterations + 1):
        r = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
        want = oracle.OPTIMAL if K == full.iterations else oracle.ITERATION_LIMIT
        assert r.status == want
        assert np.array_equal(r.trace, full.trace[:K])
        assert r.obj >= prev
        assert np.min(r.tableau[:-1, -1]) >= -1e-9
        prev = r.obj
    assert prev == full.obj
