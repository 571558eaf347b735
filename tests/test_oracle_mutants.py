"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a temporary copy of the oracle's C source
(a dropped term, a wrong sign, a wrong index, a flipped tie-break, a
transposed operand...), compiles it, and checks that at least one pin from
the same families as test_oracle_pins.py fails.  The unmodified source must
pass all of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpgen
from tests import lp_checks

SRC = os.path.join(os.path.dirname(oracle.__file__), "tableau_simplex.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")

MUTANTS = {
    "fma_sign": ("fma(-f, TAB(T, W, l, j)", "fma(f, TAB(T, W, l, j)"),
    "pricing_tie_highest": ("if (v < best) {", "if (v <= best) {"),
    "ratio_tie_highest": ("rho < best_rho", "rho <= best_rho"),
    "objective_row_skipped": ("for (int64_t i = 0; i < R; ++i) {", "for (int64_t i = 0; i < R - 1; ++i) {"),
    "negative_entries_eligible": ("if (a > eps_p) {", "if (a != 0.0) {"),
    "no_normalisation": ("TAB(T, W, l, j) = TAB(T, W, l, j) / p;", "TAB(T, W, l, j) = TAB(T, W, l, j);"),
    "slack_identity_misplaced": ("TAB(T, W, i, n + i) = 1.0;", "TAB(T, W, i, n) = 1.0;"),
    "rhs_wrong_index": ("TAB(T, W, i, W - 1) = b[i];", "TAB(T, W, i, W - 1) = b[0];"),
    "cost_sign": ("TAB(T, W, m, j) = -c[j];", "TAB(T, W, m, j) = c[j];"),
    "dual_wrong_column": ("y[i] = TAB(T, W, m, n + i);", "y[i] = TAB(T, W, m, i);"),
    "ratio_transposed": ("const double rho = r / a;", "const double rho = a / r;"),
    "pricing_skips_slacks": ("for (int64_t j = 0; j < ncols; ++j) {", "for (int64_t j = 0; j < ncols - m; ++j) {"),
    "multiplier_from_pivot_row": ("const double f = TAB(T, W, i, k);", "const double f = TAB(T, W, l, k);"),
}


def _pins(lib):
    """Return the names of the pins that fail for the library at `lib`."""
    failed = []

    def run(*a, **kw):
        return oracle.solve(*a, lib_path=lib, **kw)

    with open(GOLDEN) as f:
        for ex in json.load(f)["examples"]:
            r = run(np.array(ex["A"], float), np.array(ex["b"], float), np.array(ex["c"], float),
                    max_iter=ex.get("max_iter"))
            ok = (r.status == ex["status"] and r.trace.tolist() == ex["trace"]
                  and np.allclose(r.x, ex["x"], rtol=0, atol=1e-12)
                  and abs(r.obj - ex["obj"]) <= 1e-12 * max(1, abs(ex["obj"]))
                  and np.allclose(r.y, ex["y"], rtol=0, atol=1e-12))
            if not ok:
                failed.append("golden:" + ex["id"])
    for seed in range(6):
        rng = np.random.default_rng(1000 + seed)
        m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        A = rng.uniform(0.1, 5.0, (m, n))
        b = rng.uniform(0.0, 10.0, m)
        c = rng.uniform(-1.0, 5.0, n)
        r = run(A, b, c)
        z, _ = lp_checks.brute_force_optimum(A, b, c)
        if r.status != oracle.OPTIMAL or abs(r.obj - z) > 1e-9 * max(1.0, abs(z)):
            failed.append(f"brute:{seed}")
    A, b, c = lpgen.dense_lp(30, 20, 0)
    r = run(A, b, c, max_iter=5, want_tableau=True)
    if r.status != oracle.ITERATION_LIMIT or \
            max(lp_checks.tableau_identity_errors(A, b, c, r.basis, r.tableau).values()) > 1e-9:
        failed.append("identity")
    A, b, c = lpgen.dense_lp(64, 64, 0)
    r = run(A, b, c)
    rp, rd, gap = lp_checks.residuals(A, b, c, r.x, r.y)
    if r.status != oracle.OPTIMAL or max(rp, rd, gap) > 1e-9 or \
            abs(r.obj - lp_checks.highs_optimum(A, b, c)) > 1e-9 * abs(r.obj):
        failed.append("duality")
    return failed


def _compile(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    return oracle.build(str(src), str(tmp_path / f"lib{name}.so"))


def test_unmodified_source_passes(tmp_path):
    lib = _compile(tmp_path, "orig", open(SRC).read())
    assert _pins(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    before, after = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(before) == 1, f"mutation site for {name} not unique"
    lib = _compile(tmp_path, name, text.replace(before, after))
    assert _pins(lib), f"no pin caught the mutation {name}"
