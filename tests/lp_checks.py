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
