"""Two-phase method for general LPs (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP library.

The paper states the LP with equality rows (Section 2, eq. 1) and runs the
simplex method of Steps 1-5 from the slack basis, which needs rows A_i x <=
b_i with b >= 0.  General rows -- <=, = or >= with right-hand sides of any
sign -- take the textbook two-phase method on top of those steps.  It is
written here from its definition, G1-G9, composed of the oracle's Steps 2-5
from a basic tableau (``oracle.solve_tableau``), its pivot on a given
element (``oracle.pivot``: Steps 4-5) and its elimination of basic columns
from the objective row (``oracle.price_out``: Step 5 on the objective row):

  G1 rows       row i is multiplied by sigma_i = -1 when b_i < 0, or when
                b_i = 0 and the row reads >= (its own slack can then start
                basic); every scaled right-hand side sigma_i b_i is >= 0,
                and <= and >= swap where sigma_i = -1.
  G2 columns    Table 1's layout for the scaled rows: the n original
                variables; one surplus column (-1 in its row) per row that
                reads >=, in row order; then one column per row, in row
                order, holding the variable that starts basic in that row:
                its slack (+1) for a <= row, an artificial variable (+1) for
                a >= or = row; last the right-hand side.
  G3 phase I    maximise minus the sum of the artificial variables: in
                Table 1's sign convention the objective row holds +1 in each
                artificial column; the basic artificial columns are then
                eliminated from it (price_out), so it starts as
                -(sum of the artificial rows).
  G4            Steps 2-5 from that tableau, pricing every column.
  G5 feasible   iff phase I ends optimal with objective value (the
                objective row's RHS, minus the sum of the artificials)
                >= -1e-9 * max(1, sum of the artificial rows' scaled
                right-hand sides, added in row order); else INFEASIBLE.
  G6 drive-out  for each row in ascending order whose basic variable is
                artificial: pivot (Steps 4-5) on the lowest-index
                non-artificial column whose entry in that row has magnitude
                > eps_p; if there is none the row is redundant.
  G7 phase II   the artificial columns and the redundant rows are deleted
                (the order of the others kept); the objective row becomes
                Table 1's [-c | 0 | 0] and the basic columns are eliminated
                from it (price_out).
  G8            Steps 2-5 from that tableau, pricing every remaining column.
  G9 result     x_j = the RHS of the row whose basic variable is x_j, else
                0; z = the objective row's RHS; status of phase II;
                iterations = pivots of phase I + of the drive-out + of
                phase II.  When phase II is not reached (phase I not optimal,
                or INFEASIBLE), x is phase I's and z = sum_j c_j x_j (index
                order, multiply then add).

The iteration cap applies to each phase.  Pins: brute-force vertex
enumeration of tiny general LPs (status and optimum), an independent basis
certificate (the final basis solved with numpy: primal feasible, reduced
costs <= 0, x equal), hand-derived pivot sequences, HiGHS, and planted
mistakes that these catch (tests/test_oracle_general.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import OPTIMAL, price_out, pivot, solve_tableau

LE, EQ, GE = 0, 1, 2
INFEASIBLE = 6


@dataclass
class GeneralResult:
    status: int
    x: np.ndarray                # n original variables
    obj: float
    iterations: int              # all pivots: phase I + drive-out + phase II
    # Diagnostics (labels are the phase I columns of G2):
    trace: list = field(default_factory=list)  # (column label, original row) of every pivot, in order
    basis: np.ndarray | None = None            # final basic label of each kept row (phase II reached)
    rows: np.ndarray | None = None             # original indices of the rows kept in phase II
    phase1_iterations: int = 0
    driveout_pivots: int = 0


def row_plan(b, sense):
    """G1: sigma (+-1 per row), the scaled sense of each row, and the surplus
    column of each row that reads >= after scaling (-1 elsewhere)."""
    m = b.shape[0]
    sigma = np.ones(m)
    scaled = np.zeros(m, dtype=np.int8)
    surcol = np.full(m, -1, dtype=np.int64)
    q = 0
    for i in range(m):
        s = LE if sense is None else int(sense[i])
        bi = float(b[i])
        flip = bi < 0.0 or (bi == 0.0 and s == GE)
        sigma[i] = -1.0 if flip else 1.0
        scaled[i] = {LE: GE, GE: LE, EQ: EQ}[s] if flip else s
        if scaled[i] == GE:
            surcol[i] = q
            q += 1
    return sigma, scaled, surcol, q


def phase1_tableau(A, b, sense):
    """G1-G3: the phase I tableau and its starting basis (column labels)."""
    m, n = A.shape
    sigma, scaled, surcol, q = row_plan(b, sense)
    n1 = n + q
    W = n1 + m + 1
    T = np.zeros((m + 1, W))
    art = scaled != LE
    for i in range(m):
        T[i, :n] = sigma[i] * A[i]
        if surcol[i] >= 0:
            T[i, n + surcol[i]] = -1.0
        T[i, n1 + i] = 1.0
        T[i, W - 1] = sigma[i] * b[i]
        if art[i]:
            T[m, n1 + i] = 1.0
    basis = n1 + np.arange(m, dtype=np.int64)
    price_out(T, basis)
    return T, basis, n1, art, sigma, scaled, surcol


def _dot_in_order(c, x):
    acc = 0.0
    for j in range(c.shape[0]):
        acc = acc + float(c[j]) * float(x[j])
    return acc


def solve_general(A, b, c, sense=None, *, eps_d: float = 1e-9, eps_p: float = 1e-9,
                  max_iter: int | None = None, lib_path: str | None = None) -> GeneralResult:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1)
    m, n = A.shape
    if max_iter is None:
        max_iter = 50 * (m + n)
    T1, basis1, n1, art, sigma, _, _ = phase1_tableau(A, b, sense)
    ncols1 = n1 + m

    # G4: phase I.
    r1 = solve_tableau(T1, basis1, eps_d=eps_d, eps_p=eps_p, max_iter=max_iter, lib_path=lib_path)
    trace = [(int(k), int(l)) for k, l in r1.trace]
    it1 = r1.iterations
    sum_b_art = 0.0
    for i in range(m):
        if art[i]:
            sum_b_art = sum_b_art + float(sigma[i] * b[i])
    feasible = r1.status == OPTIMAL and r1.obj >= -1e-9 * max(1.0, sum_b_art)
    if not feasible:
        status = INFEASIBLE if r1.status == OPTIMAL else r1.status
        x = r1.x[:n].copy()
        return GeneralResult(status, x, _dot_in_order(c, x), it1, trace, phase1_iterations=it1)

    # G6: drive the artificial variables out of the basis.
    T = r1.tableau.copy()
    basis = r1.basis.copy()
    is_art = np.zeros(ncols1, dtype=bool)
    is_art[n1:] = art
    redundant = []
    nd = 0
    for i in range(m):
        if not is_art[basis[i]]:
            continue
        cols = [j for j in range(ncols1) if not is_art[j] and abs(T[i, j]) > eps_p]
        if cols:
            j = cols[0]
            pivot(T, i, j, lib_path=lib_path)
            basis[i] = j
            trace.append((j, i))
            nd += 1
        else:
            redundant.append(i)

    # G7: phase II tableau.
    rows = np.array([i for i in range(m) if i not in redundant], dtype=np.int64)
    cols = np.array([j for j in range(ncols1) if not is_art[j]], dtype=np.int64)
    T2 = np.ascontiguousarray(T[np.append(rows, m)][:, np.append(cols, ncols1)])
    where = {int(j): t for t, j in enumerate(cols)}
    basis2 = np.array([where[int(basis[i])] for i in rows], dtype=np.int64)
    m2 = rows.shape[0]
    T2[m2, :] = 0.0
    T2[m2, :n] = -c  # the first n kept columns are the original variables
    price_out(T2, basis2)

    # G8: phase II.
    r2 = solve_tableau(T2, basis2, eps_d=eps_d, eps_p=eps_p, max_iter=max_iter, lib_path=lib_path)
    trace += [(int(cols[k]), int(rows[l])) for k, l in r2.trace]

    # G9.
    x = np.zeros(n)
    for i, v in enumerate(r2.basis):
        if cols[v] < n:
            x[cols[v]] = r2.tableau[i, -1]
    return GeneralResult(r2.status, x, r2.obj, it1 + nd + r2.iterations, trace,
                         basis=cols[r2.basis], rows=rows, phase1_iterations=it1, driveout_pivots=nd)
