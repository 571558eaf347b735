"""Reference for general LPs, two-phase method (test infrastructure only).

Only the tests may import this module.  It composes the paper-method oracle
(``oracle.solve``: Steps 1-5 of Section 2 from the slack basis of a <= LP
with b >= 0) with the textbook two-phase construction, step by step in plain
numpy, so that the GPU library's lp_solve_general can be compared with it bit
for bit.  The construction (the paper assumes b >= 0 and does not need it):

  row plan   each row is scaled by sigma = +-1 so that its right-hand side is
             >= 0: "<=" with b >= 0 stays; "<=" with b < 0 and ">=" with
             b > 0 become ">=" rows (surplus column, artificial basic);
             ">=" with b <= 0 becomes a "<=" row; "=" rows get an artificial.
  phase I    max c1^T x1, A1 x1 <= b1 (the artificial is the row's slack),
             c1 = sum of the artificial rows of A1 (rows in order); feasible
             iff the optimum reaches the sum of their b1 (rel. tol. 1e-9).
  phase II   the nonbasic non-artificial columns of phase I's final tableau,
             b2 = max(rhs, +0) (0 where an artificial stayed basic, plus a
             mirrored row for it), costs c_N - sum_i c_B[i] A2[i] (rows in
             order, separate multiply and add).
  recover    nonbasic variables from phase II's x; a variable basic in row i
             from b2[i] - sum_u A2[i, u] x2[u] (columns in order);
             obj = sum_j c[j] x[j] (index order).

Pins: objective and feasibility against scipy's HiGHS, infeasible and
unbounded cases, and the reduction to ``oracle.solve`` when no row needs an
artificial (tests/test_oracle_general.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import solve as _solve, OPTIMAL

LE, EQ, GE = 0, 1, 2
INFEASIBLE = 6


@dataclass
class GeneralResult:
    status: int
    x: np.ndarray
    obj: float
    iterations: int


def _row_plan(b, sense):
    m = b.shape[0]
    sigma = np.ones(m)
    art = np.zeros(m, dtype=bool)
    surcol = np.full(m, -1)
    q = 0
    for i in range(m):
        s = LE if sense is None else int(sense[i])
        bi = b[i]
        if s == LE:
            if bi < 0.0:
                sigma[i], art[i], surcol[i] = -1.0, True, q
                q += 1
        elif s == GE:
            if bi > 0.0:
                art[i], surcol[i] = True, q
                q += 1
            else:
                sigma[i] = -1.0
        else:
            sigma[i] = -1.0 if bi < 0.0 else 1.0
            art[i] = True
    return sigma, art, surcol, q


def _dot_in_order(c, x):
    acc = 0.0
    for j in range(c.shape[0]):
        acc = acc + float(c[j]) * float(x[j])
    return acc


def solve_general(A, b, c, sense=None, *, eps_d: float = 1e-9, eps_p: float = 1e-9,
                  max_iter: int | None = None) -> GeneralResult:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    m, n = A.shape
    sigma, art, surcol, q = _row_plan(b, sense)
    n1 = n + q
    A1 = np.zeros((m, n1))
    A1[:, :n] = np.where(sigma[:, None] > 0, A, -A)
    for i in range(m):
        if surcol[i] >= 0:
            A1[i, n + surcol[i]] = -1.0
    b1 = np.abs(b)
    n_art = int(art.sum())
    if n_art:
        c1 = np.zeros(n1)
        for i in range(m):
            if art[i]:
                c1 = c1 + A1[i]
    else:
        c1 = c.copy()
    sum_b_art = 0.0
    for i in range(m):
        if art[i]:
            sum_b_art = sum_b_art + abs(float(b[i]))

    r1 = _solve(A1, b1, c1, eps_d=eps_d, eps_p=eps_p, max_iter=max_iter, want_tableau=n_art > 0)
    feasible = r1.status == OPTIMAL and (n_art == 0 or r1.obj >= sum_b_art - 1e-9 * max(1.0, sum_b_art))
    if n_art == 0 or r1.status != OPTIMAL or not feasible:
        status = INFEASIBLE if (r1.status == OPTIMAL and not feasible) else r1.status
        x = r1.x[:n].copy()
        return GeneralResult(status, x, _dot_in_order(c, x), r1.iterations)

    T1 = r1.tableau
    basis1 = r1.basis.astype(np.int64)
    basic = np.zeros(n1 + m, dtype=bool)
    basic[basis1] = True
    is_art = np.zeros(n1 + m, dtype=bool)
    is_art[n1:] = art
    N = np.array([v for v in range(n1 + m) if not basic[v] and not is_art[v]], dtype=np.int64)
    extra = [i for i in range(m) if is_art[basis1[i]]]
    cost = np.zeros(n1 + m)
    cost[:n] = c
    cB = cost[basis1]
    cN = cost[N]
    n2 = N.shape[0]
    rhs = T1[:m, -1]
    b2 = np.where(rhs > 0.0, rhs, 0.0)
    b2[extra] = 0.0
    A2 = T1[:m][:, N]
    if extra:
        A2 = np.vstack([A2, -T1[extra][:, N]])
        b2 = np.concatenate([b2, np.zeros(len(extra))])
    it2, st2, x2 = 0, OPTIMAL, np.zeros(0)
    if n2:
        acc = np.zeros(n2)
        for i in range(m):
            acc = acc + cB[i] * A2[i]
        c2 = cN - acc
        r2 = _solve(A2, b2, c2, eps_d=eps_d, eps_p=eps_p, max_iter=max_iter)
        it2, st2, x2 = r2.iterations, r2.status, r2.x
    x = np.zeros(n)
    for t in range(n2):
        if N[t] < n:
            x[N[t]] = x2[t]
    acc = np.zeros(m)
    for u in range(n2):
        acc = acc + A2[:m, u] * x2[u]
    for i in range(m):
        if basis1[i] < n:
            x[basis1[i]] = b2[i] - acc[i]
    return GeneralResult(st2, x, _dot_in_order(c, x), r1.iterations + it2)
