"""Checks that pin an LP solution to the mathematics, independently of any
solver under test: brute-force vertex enumeration, an LP library (HiGHS via
scipy), feasibility and duality residuals, and the textbook identities a
simplex tableau must satisfy for its current basis."""
from __future__ import annotations

import itertools

import numpy as np


def brute_force_optimum(A, b, c):
    """max c^T x s.t. Ax <= b, x >= 0 by enumerating every basis of [A | I].

    Only for tiny bounded LPs (C(n+m, m) bases).  Returns (z*, x*)."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = np.hstack([A, np.eye(m)])
    cext = np.concatenate([np.asarray(c, float), np.zeros(m)])
    best, bx = -np.inf, None
    for S in itertools.combinations(range(n + m), m):
        B = M[:, S]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        zS = np.linalg.solve(B, b)
        if np.all(zS >= -1e-9):
            val = float(cext[list(S)] @ zS)
            if val > best:
                best = val
                z = np.zeros(n + m)
                z[list(S)] = zS
                bx = z[:n]
    return best, bx


def highs_optimum(A, b, c):
    from scipy.optimize import linprog
    res = linprog(-np.asarray(c, float), A_ub=A, b_ub=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return -float(res.fun)


def residuals(A, b, c, x, y):
    """Scaled residuals: primal infeasibility, dual infeasibility, duality gap."""
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    rp = max(float(np.max(np.maximum(A @ x - b, 0.0), initial=0.0)),
             float(np.max(np.maximum(-x, 0.0), initial=0.0))) / (1.0 + float(np.max(np.abs(b))))
    rd = max(float(np.max(np.maximum(c - A.T @ y, 0.0), initial=0.0)),
             float(np.max(np.maximum(-y, 0.0), initial=0.0))) / (1.0 + float(np.max(np.abs(c))))
    px, dy = float(c @ x), float(b @ y)
    gap = abs(px - dy) / max(1.0, abs(px))
    return rp, rd, gap


def complementary_slackness(A, b, c, x, y, tol=1e-7):
    """max over i of |y_i (b - Ax)_i| and over j of |x_j (A^T y - c)_j|, scaled."""
    A = np.asarray(A, float)
    s = b - A @ x
    d = A.T @ y - c
    scale = (1.0 + np.max(np.abs(b))) * (1.0 + np.max(np.abs(c)))
    return max(float(np.max(np.abs(y * s))), float(np.max(np.abs(x * d)))) / scale


def tableau_identity_errors(A, b, c, basis, T):
    """Compare a tableau with the textbook formulas for its basis B (columns of
    [A | I] listed by `basis`, row i <-> basis[i]):
      T[:m, :n] = B^-1 A,  T[:m, n:n+m] = B^-1,  T[:m, -1] = B^-1 b,
      T[m, :n] = c_B B^-1 A - c,  T[m, n:n+m] = c_B B^-1,  T[m, -1] = c_B B^-1 b.
    Returns the max abs error of each block divided by its scale."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = np.hstack([A, np.eye(m)])
    cext = np.concatenate([np.asarray(c, float), np.zeros(m)])
    B = M[:, basis]
    Binv = np.linalg.inv(B)
    cB = cext[basis]
    want_body = Binv @ M
    want_rhs = Binv @ b
    want_obj = cB @ want_body - cext
    want_z = float(cB @ want_rhs)
    errs = {
        "body": np.max(np.abs(T[:m, : n + m] - want_body)) / (1.0 + np.max(np.abs(want_body))),
        "rhs": np.max(np.abs(T[:m, -1] - want_rhs)) / (1.0 + np.max(np.abs(want_rhs))),
        "obj": np.max(np.abs(T[m, : n + m] - want_obj)) / (1.0 + np.max(np.abs(want_obj))),
        "z": abs(T[m, -1] - want_z) / (1.0 + abs(want_z)),
    }
    return errs


# ---------------------------------------------------------------------------
# General LPs: rows A_i x (<=, =, >=) b_i with sense codes 0, 1, 2; x >= 0.

def _general_feasible(A, b, sense, x, tol):
    ax = A @ x
    scale = 1.0 + float(np.max(np.abs(b), initial=0.0))
    ok = np.all(x >= -tol * scale)
    ok &= np.all(ax[sense == 0] <= b[sense == 0] + tol * scale)
    ok &= np.all(ax[sense == 2] >= b[sense == 2] - tol * scale)
    ok &= np.all(np.abs(ax[sense == 1] - b[sense == 1]) <= tol * scale)
    return bool(ok)


def _general_vertices(A, b, sense, box=None, tol=1e-9):
    """Feasible vertices of {x >= 0, A_i x (sense_i) b_i} (and sum(x) <= box):
    every choice of n linearly independent active constraints among the rows,
    the bounds x_j = 0 and the box, kept if feasible."""
    m, n = A.shape
    planes = [(A[i], b[i]) for i in range(m)] + [(np.eye(n)[j], 0.0) for j in range(n)]
    if box is not None:
        planes.append((np.ones(n), box))
    out = []
    for S in itertools.combinations(range(len(planes)), n):
        M = np.array([planes[s][0] for s in S])
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, np.array([planes[s][1] for s in S]))
        if _general_feasible(A, b, sense, x, tol) and (box is None or x.sum() <= box * (1 + 1e-12)):
            out.append(x)
    return out


def brute_force_general(A, b, c, sense):
    """Status and optimum of max c^T x over a tiny general LP by vertex
    enumeration: 'infeasible' if there is no feasible vertex (a nonempty
    polyhedron inside x >= 0 has one), 'unbounded' if the best vertex value
    keeps growing when the box sum(x) <= M grows from 1e5 to 1e7, else
    'optimal' with z* and the vertices that attain it."""
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    sense = np.asarray(sense)
    vs = _general_vertices(A, b, sense)
    if not vs:
        return "infeasible", None, []
    best = max(float(c @ v) for v in vs)
    big1 = max(float(c @ v) for v in _general_vertices(A, b, sense, box=1e5))
    big2 = max(float(c @ v) for v in _general_vertices(A, b, sense, box=1e7))
    if big2 > big1 + 1e-6 * max(1.0, abs(big1)):
        return "unbounded", None, []
    at = [v for v in vs if abs(float(c @ v) - best) <= 1e-9 * max(1.0, abs(best))]
    return "optimal", best, at


def general_basis_certificate(A, b, c, sense, labels, rows):
    """Checks a final basis of the two-phase method without its tableau.

    The LP in equality form has one slack u_i >= 0 per inequality row:
    A_i x + u_i = b_i (<=) or A_i x - u_i = b_i (>=).  The method's column
    labels are: 0..n-1 the x_j; then one surplus column per row that reads >=
    after multiplying the rows with b_i < 0 (or b_i = 0 and >=) by -1, in row
    order; then n1 + i for row i's own column (its slack where the row then
    reads <=).  Either way the column is u_i of the original row.  With B the
    basic columns of [A | U] over the kept rows, x_B = B^-1 b must be >= 0 and
    satisfy every row (the deleted ones too), and y = B^-T c_B must leave no
    positive reduced cost c_j - a_j^T y.  Returns (x, dict of scaled errors)."""
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    sense = np.asarray(sense)
    m, n = A.shape
    flip = (b < 0) | ((b == 0) & (sense == 2))
    scaled = np.where(flip, np.select([sense == 0, sense == 2], [2, 0], 1), sense)
    ge_rows = [i for i in range(m) if scaled[i] == 2]
    n1 = n + len(ge_rows)
    col_of_label = {j: j for j in range(n)}
    for t, i in enumerate(ge_rows):
        col_of_label[n + t] = n + i       # u_i
    for i in range(m):
        if scaled[i] == 0:
            col_of_label[n1 + i] = n + i  # u_i
    U = np.zeros((m, m))
    for i in range(m):
        U[i, i] = {0: 1.0, 2: -1.0, 1: 0.0}[int(sense[i])]
    E = np.hstack([A, U])
    cost = np.concatenate([c, np.zeros(m)])
    cols = [col_of_label[int(v)] for v in labels]
    rows = np.asarray(rows, dtype=np.int64)
    B = E[rows][:, cols]
    vB = np.linalg.solve(B, b[rows])
    v = np.zeros(n + m)
    v[cols] = vB
    x = v[:n]
    y = np.linalg.solve(B.T, cost[cols])
    usable = [j for j in range(n + m) if j < n or int(sense[j - n]) != 1]
    red = cost[usable] - E[rows][:, usable].T @ y
    res = E @ v - b
    scale_b = 1.0 + float(np.max(np.abs(b)))
    errs = {
        "primal_negative": float(max(0.0, -np.min(v))) / scale_b,
        "rows_violated": float(np.max(np.abs(res))) / scale_b,
        "reduced_cost_positive": float(max(0.0, np.max(red))) / (1.0 + float(np.max(np.abs(c)))),
    }
    return x, errs
