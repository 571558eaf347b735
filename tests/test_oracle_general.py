"""Pins of the two-phase reference (oracle/general.py) to things other than
itself (CPU only): hand-derived pivot sequences, brute-force vertex
enumeration of tiny general LPs (every status), an independent basis
certificate (numpy solves with the final basis), scipy's HiGHS, the exact
reduction to the paper-method oracle when no row needs an artificial
variable, and planted mistakes that these pins catch."""
import json
import os
import sys
import types

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from oracle import general
from paper_1804_04737_amd import lpgen
from tests import lp_checks
from tests.gpu_util import bits

HERE = os.path.dirname(os.path.abspath(__file__))
EXAMPLES = os.path.join(HERE, "golden", "general_examples.json")
STATUS = {"optimal": oracle.OPTIMAL, "unbounded": oracle.UNBOUNDED, "infeasible": general.INFEASIBLE}


def _examples():
    with open(EXAMPLES) as f:
        return json.load(f)["examples"]


def _highs(A, b, c, sense):
    le, eq, ge = sense == 0, sense == 1, sense == 2
    A_ub = np.vstack([A[le], -A[ge]])
    b_ub = np.concatenate([b[le], -b[ge]])
    return linprog(-c, A_ub=A_ub if len(A_ub) else None, b_ub=b_ub if len(b_ub) else None,
                   A_eq=A[eq] if eq.any() else None, b_eq=b[eq] if eq.any() else None,
                   bounds=[(0, None)] * A.shape[1], method="highs")


def _tiny(seed):
    """A tiny general LP with integer data: rows of every sense, right-hand
    sides of both signs (zeros included), repeated rows now and then."""
    rng = np.random.default_rng(7000 + seed)
    m, n = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    A = rng.integers(-4, 6, (m, n)).astype(float)
    b = rng.integers(-6, 9, m).astype(float)
    c = rng.integers(-3, 6, n).astype(float)
    sense = rng.integers(0, 3, m).astype(np.int8)
    if m >= 2 and seed % 5 == 0:  # a repeated equality row: redundant after phase I
        A[1], b[1], sense[0], sense[1] = A[0], b[0], 1, 1
    if seed % 7 == 3:
        b[rng.integers(0, m)] = 0.0
    return A, b, c, sense


def _tiny_tie(seed):
    """A tiny general LP whose row 1 restates row 0 (a <= row) as an
    equality: phase I's ratio test ties the two rows, the lower one leaves,
    and row 1's artificial variable stays basic at level zero -- the case of
    the drive-out pivot."""
    rng = np.random.default_rng(9000 + seed)
    m, n = int(rng.integers(2, 5)), int(rng.integers(1, 5))
    A = rng.integers(-4, 6, (m, n)).astype(float)
    b = rng.integers(-6, 9, m).astype(float)
    c = rng.integers(-3, 6, n).astype(float)
    sense = rng.integers(0, 3, m).astype(np.int8)
    A[0] = np.abs(A[0]) + 1
    b[0] = abs(b[0]) + 1
    A[1], b[1], sense[0], sense[1] = A[0], b[0], 0, 1
    return A, b, c, sense


def _tiny_cases(count):
    return [_tiny(s) for s in range(count)] + [_tiny_tie(s) for s in range(count // 2)]


def _pins(gen, seeds=range(60), basis_cases=True):
    """Names of the pins the module `gen` fails (empty: all pass).  A pin
    whose check cannot even be evaluated on the result (no basis returned, an
    artificial variable in the final basis, ...) fails too."""
    failed = []

    def pin(name, check):
        try:
            if not check():
                failed.append(name)
        except Exception as e:  # noqa: BLE001 - the result is not what the pin describes
            failed.append(f"{name} ({type(e).__name__})")

    def example_ok(ex):
        r = gen.solve_general(np.array(ex["A"], float), np.array(ex["b"], float), np.array(ex["c"], float),
                              np.array(ex["sense"], np.int8))
        return (r.status == ex["status"] and r.iterations == ex["iterations"]
                and [list(t) for t in r.trace] == ex["trace"]
                and r.phase1_iterations == ex["phase1_iterations"] and r.driveout_pivots == ex["driveout_pivots"]
                and np.array_equal(r.x, np.array(ex["x"], float)) and r.obj == ex["obj"]
                and list(r.rows) == ex["rows"])

    for ex in _examples():
        pin("example:" + ex["id"], lambda ex=ex: example_ok(ex))
    for seed, (A, b, c, sense) in enumerate([_tiny(s) for s in seeds] + [_tiny_tie(s) for s in range(20)]):
        want, z, at = lp_checks.brute_force_general(A, b, c, sense)
        r = gen.solve_general(A, b, c, sense)
        pin(f"brute_status:{seed}", lambda: r.status == STATUS[want])
        if want == "optimal" and r.status == STATUS[want]:
            pin(f"brute_optimum:{seed}", lambda: abs(r.obj - z) <= 1e-9 * max(1.0, abs(z))
                and any(np.allclose(r.x, v, atol=1e-9) for v in at))
            pin(f"certificate:{seed}", lambda: max(lp_checks.general_basis_certificate(
                A, b, c, sense, r.basis, r.rows)[1].values()) <= 1e-9)
    if basis_cases:
        for m, n, seed in [(20, 15, 3), (40, 60, 4), (120, 90, 5)]:
            A, b, c, sense = lpgen.general_lp(m, n, seed)
            r = gen.solve_general(A, b, c, sense)

            def cert_ok():
                x_cert, errs = lp_checks.general_basis_certificate(A, b, c, sense, r.basis, r.rows)
                return (r.status == oracle.OPTIMAL and max(errs.values()) <= 1e-9
                        and np.max(np.abs(x_cert - r.x)) <= 1e-9 * (1 + np.max(np.abs(r.x))))
            pin(f"certificate_generator:{m}x{n}", cert_ok)
    return failed


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["id"])
def test_hand_derived_examples(ex):
    r = general.solve_general(np.array(ex["A"], float), np.array(ex["b"], float), np.array(ex["c"], float),
                              np.array(ex["sense"], np.int8))
    assert r.status == ex["status"]
    assert [list(t) for t in r.trace] == ex["trace"]
    assert r.iterations == ex["iterations"]
    assert (r.phase1_iterations, r.driveout_pivots) == (ex["phase1_iterations"], ex["driveout_pivots"])
    assert list(r.rows) == ex["rows"]
    assert np.array_equal(r.x, np.array(ex["x"], float)) and r.obj == ex["obj"]


@pytest.mark.parametrize("case", range(180))
def test_brute_force_tiny_general(case):
    """Status (optimal / unbounded / infeasible) and optimum equal vertex
    enumeration; an optimal x is an optimal vertex; its basis certifies it."""
    A, b, c, sense = _tiny(case) if case < 120 else _tiny_tie(case - 120)
    want, z, at = lp_checks.brute_force_general(A, b, c, sense)
    r = general.solve_general(A, b, c, sense)
    assert r.status == STATUS[want], (want, r.status)
    if want == "optimal":
        assert abs(r.obj - z) <= 1e-9 * max(1.0, abs(z))
        assert any(np.allclose(r.x, v, atol=1e-9) for v in at)
        x_cert, errs = lp_checks.general_basis_certificate(A, b, c, sense, r.basis, r.rows)
        assert max(errs.values()) <= 1e-9, errs
        assert np.allclose(x_cert, r.x, atol=1e-9)


def test_tiny_cases_cover_every_outcome():
    """The tiny set above meets all three statuses, drive-out pivots and
    redundant rows, so each branch of G5-G7 is pinned."""
    seen, drive, redundant = set(), 0, 0
    for A, b, c, sense in _tiny_cases(120):
        r = general.solve_general(A, b, c, sense)
        seen.add(r.status)
        drive += r.driveout_pivots
        if r.rows is not None and len(r.rows) < A.shape[0]:
            redundant += 1
    assert {oracle.OPTIMAL, oracle.UNBOUNDED, general.INFEASIBLE} <= seen
    assert drive > 0 and redundant > 0


@pytest.mark.parametrize("m,n,seed", [(3, 4, 0), (5, 5, 1), (8, 12, 2), (20, 15, 3), (40, 60, 4), (120, 90, 5)])
def test_general_matches_highs_and_certificate(m, n, seed):
    A, b, c, sense = lpgen.general_lp(m, n, seed)
    r = general.solve_general(A, b, c, sense)
    h = _highs(A, b, c, sense)
    assert h.status == 0 and r.status == oracle.OPTIMAL
    assert abs(r.obj - (-h.fun)) <= 1e-9 * max(1.0, abs(h.fun))
    x_cert, errs = lp_checks.general_basis_certificate(A, b, c, sense, r.basis, r.rows)
    assert max(errs.values()) <= 1e-9, errs
    assert np.max(np.abs(x_cert - r.x)) <= 1e-9 * (1 + np.max(np.abs(r.x)))


def test_reduces_to_the_paper_method_without_artificials():
    """Only <= rows with b >= 0 (or >= rows with b <= 0): phase I has no
    artificial, ends at once, and phase II is Table 1 itself, so the result
    is the paper-method oracle's bit for bit."""
    A, b, c = lpgen.dense_lp(30, 40, 9)
    for AA, bb, sense in ((A, b, None), (-A, -b, np.full(30, 2, np.int8))):
        r = general.solve_general(AA, bb, c, sense)
        ref = oracle.solve(A, b, c)
        assert r.status == ref.status and r.iterations == ref.iterations
        assert [list(t) for t in r.trace] == ref.trace.tolist()
        assert np.array_equal(bits(r.x), bits(ref.x)) and bits([r.obj])[0] == bits([ref.obj])[0]


def test_infeasible_unbounded_and_degenerate_cases():
    A = np.array([[1.0, 1.0], [1.0, 0.0]])
    c = np.array([1.0, 1.0])
    r = general.solve_general(A, np.array([-1.0, 5.0]), c, np.array([1, 0], np.int8))
    assert r.status == general.INFEASIBLE and abs(r.obj - float(c @ r.x)) <= 1e-12 * (1 + abs(r.obj))
    for seed in range(120):  # z of every infeasible tiny LP is c^T x of the point returned
        A, b, cc, sense = _tiny(seed)
        r = general.solve_general(A, b, cc, sense)
        if r.status == general.INFEASIBLE:
            assert abs(r.obj - float(cc @ r.x)) <= 1e-12 * (1 + np.abs(cc).sum() * (1 + np.abs(r.x).max()))
    r = general.solve_general(np.eye(2), np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([2, 2], np.int8))
    assert r.status == oracle.UNBOUNDED
    # A square nonsingular equality system: every original variable basic.
    r = general.solve_general(np.array([[2.0, 1.0], [1.0, 3.0]]), np.array([5.0, 10.0]), np.array([1.0, 1.0]),
                              np.array([1, 1], np.int8))
    assert r.status == oracle.OPTIMAL and np.allclose(r.x, [1.0, 3.0], atol=1e-12)
    # Every row redundant: no constraint row left for phase II.
    r = general.solve_general(np.zeros((2, 2)), np.zeros(2), np.array([1.0, -1.0]), np.array([1, 1], np.int8))
    assert r.status == oracle.UNBOUNDED and len(r.rows) == 0
    r = general.solve_general(np.zeros((2, 2)), np.zeros(2), np.array([-1.0, -1.0]), np.array([1, 1], np.int8))
    assert r.status == oracle.OPTIMAL and np.all(r.x == 0)
    # NaN: the phase I tableau is not finite.
    A, b, c, sense = lpgen.general_lp(10, 10, 1)
    A[3, 4] = np.nan
    assert general.solve_general(A, b, c, sense).status == oracle.NUMERICAL


# Planted mistakes in a copy of general.py: each must make some pin fail.
MUTANTS = {
    "surplus_sign": ("T[i, n + surcol[i]] = -1.0", "T[i, n + surcol[i]] = 1.0"),
    "phase1_objective_sign": ("T[m, n1 + i] = 1.0", "T[m, n1 + i] = -1.0"),
    "no_phase1_price_out": ("    price_out(T, basis)\n    return T, basis", "    return T, basis"),
    "phase2_cost_sign": ("T2[m2, :n] = -c", "T2[m2, :n] = c"),
    "no_phase2_price_out": ("    price_out(T2, basis2)\n", ""),
    "feasibility_test_flipped": ("r1.obj >= -1e-9 * max(1.0, sum_b_art)", "r1.obj <= -1e-9 * max(1.0, sum_b_art)"),
    "artificials_kept_in_phase2": ("if not is_art[j]], dtype=np.int64)", "], dtype=np.int64)"),
    "no_drive_out": ("        if cols:\n", "        if False:\n"),
    "drive_out_on_artificial": ("if not is_art[j] and abs(T[i, j]) > eps_p]", "if abs(T[i, j]) > eps_p]"),
    "rhs_not_scaled": ("T[i, W - 1] = sigma[i] * b[i]", "T[i, W - 1] = b[i]"),
    "flip_rule_b_zero": ("flip = bi < 0.0 or (bi == 0.0 and s == GE)", "flip = bi <= 0.0"),
}


def _mutant_module(name, text):
    mod = types.ModuleType(f"oracle._mutant_{name}")
    mod.__package__ = "oracle"
    mod.__file__ = general.__file__
    sys.modules[mod.__name__] = mod
    try:
        exec(compile(text, f"<mutant {name}>", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


def test_unmodified_reference_passes_the_pins():
    assert _pins(general) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    before, after = MUTANTS[name]
    text = open(general.__file__).read()
    assert text.count(before) == 1, f"mutation site for {name} not unique"
    mod = _mutant_module(name, text.replace(before, after))
    try:
        failed = _pins(mod)
    except Exception as e:  # noqa: BLE001 - a mistake that breaks the method outright is caught too
        failed = [f"solve_general raised {type(e).__name__}"]
    assert failed, f"no pin caught the planted mistake {name}"
