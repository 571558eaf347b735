"""Seeded synthetic LP workloads (inputs only; no simplex arithmetic here).

Both the HIP library's tests/benchmarks and the reference oracle draw their
inputs from this module, so it holds nothing but random-number draws.

Dense generator G(m, n, seed), for  max c^T x  s.t.  A x <= b,  x >= 0:
    rng = numpy.random.default_rng(seed)          (PCG64)
    A   = rng.integers(1, 101, (m, n))  as float64 (integer uniform [1, 100])
    b   = rng.uniform(1000 s, 10000 s, m), s = n / 64
    c   = rng.integers(1, 101, n)       as float64
drawn in that order.  A > 0 and b > 0 make every instance feasible at x = 0
and bounded.  It stands in for the paper's own random instances, which are
not available (Section 4 describes dense random problems of sizes 256..8192).
"""
from __future__ import annotations

import math

import numpy as np


def dense_lp(m: int, n: int, seed: int):
    """One dense LP (A, b, c) with the distribution described above."""
    rng = np.random.default_rng(seed)
    A = rng.integers(1, 101, size=(m, n)).astype(np.float64)
    s = n / 64.0
    b = rng.uniform(1000.0 * s, 10000.0 * s, size=m)
    c = rng.integers(1, 101, size=n).astype(np.float64)
    return A, b, c


def log_uniform_int(rng, lo: int, hi: int, size=None):
    """round(exp(U(ln lo, ln hi))) clipped to [lo, hi]."""
    v = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)
    return np.clip(v, lo, hi)


def batch_shapes(count: int, lo: int, hi: int, seed: int = 0):
    """Shapes (m_i, n_i), each independently log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    m = log_uniform_int(rng, lo, hi, size=count)
    n = log_uniform_int(rng, lo, hi, size=count)
    return m, n


def batch_lps(count: int, lo: int = 32, hi: int = 1024, seed: int = 0):
    """A batch of independent dense LPs of uneven sizes.

    Shapes come from `batch_shapes(count, lo, hi, seed)`; instance i then uses
    dense_lp(m_i, n_i, seed_i) with seed_i the i-th child of
    numpy.random.SeedSequence(seed).
    """
    m, n = batch_shapes(count, lo, hi, seed)
    children = np.random.SeedSequence(seed).spawn(count)
    return [dense_lp(int(m[i]), int(n[i]), _child_seed(children[i])) for i in range(count)]


def _child_seed(child) -> int:
    return int(child.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1))


def batch_lp(i: int, count: int, lo: int = 32, hi: int = 1024, seed: int = 0):
    """Instance i of `batch_lps(count, lo, hi, seed)`, drawn on its own."""
    m, n = batch_shapes(count, lo, hi, seed)
    child = np.random.SeedSequence(seed).spawn(count)[i]
    return dense_lp(int(m[i]), int(n[i]), _child_seed(child))


def poisson_arrivals(rate: float, count: int, seed: int = 0):
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# The paper's experiments (Section 4) use problem shapes m, n in this set.
PAPER_SIZES = (256, 512, 1024, 2048, 4096, 8192)


def paper_lp(m: int, n: int, seed: int, density: float = 0.9):
    """A second workload with the behaviour of the paper's random generator
    (Section 4): a dense-ish A with about `density` of its entries nonzero,
    values between 0 and 50, and b built from a random non-negative point so
    that every instance is feasible.  Written from that description (the
    printed listing is garbled and is not reproduced); integer values keep
    every draw, b and c exact on any machine:

        rng  = numpy.random.default_rng(seed)
        mask = rng.random((m, n)) < density
        A    = mask * rng.integers(1, 51, (m, n))       (float64)
        x0   = rng.integers(0, 11, n)                    (a point with A x0 = b)
        b    = A @ x0                                    (exact: integers < 2^53)
        repeat: u = rng.integers(-1, 2, m); c = A^T u    until some c_j > 0

    A >= 0 with no empty column (almost surely) keeps max c^T x bounded; x0
    and x = 0 are feasible.  c has both signs, so pricing meets many ties and
    zero reduced costs, unlike dense_lp.
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    A = (mask * rng.integers(1, 51, (m, n))).astype(np.float64)
    x0 = rng.integers(0, 11, n).astype(np.float64)
    b = A @ x0
    while True:
        u = rng.integers(-1, 2, m).astype(np.float64)
        c = A.T @ u
        if np.any(c > 0):
            return A, b, c


def general_lp(m: int, n: int, seed: int, p_eq: float = 0.2, p_ge: float = 0.3, bounded: bool = True):
    """A general LP for the two-phase path: rows of every sense and
    right-hand sides of both signs, feasible by construction at a point x0.

        rng   = numpy.random.default_rng(seed)
        A     = rng.integers(-10, 11, (m, n))      (float64)
        x0    = rng.integers(0, 6, n)
        slack = rng.integers(0, 6, m)
        sense = LE / EQ / GE with probabilities 1-p_eq-p_ge, p_eq, p_ge
        b     = A x0 + slack (LE), A x0 (EQ), A x0 - slack (GE)
        c     = rng.integers(-5, 11, n)
    With bounded=True the last row is replaced by sum(x) <= sum(x0) + 10 (LE),
    which keeps the optimum finite.  Returns (A, b, c, sense) with sense as
    int8 codes 0 (<=), 1 (=), 2 (>=).
    """
    rng = np.random.default_rng(seed)
    A = rng.integers(-10, 11, (m, n)).astype(np.float64)
    x0 = rng.integers(0, 6, n).astype(np.float64)
    slack = rng.integers(0, 6, m).astype(np.float64)
    u = rng.random(m)
    sense = np.where(u < p_eq, 1, np.where(u < p_eq + p_ge, 2, 0)).astype(np.int8)
    ax = A @ x0
    b = np.where(sense == 0, ax + slack, np.where(sense == 2, ax - slack, ax))
    c = rng.integers(-5, 11, n).astype(np.float64)
    if bounded:
        A[-1] = 1.0
        b[-1] = x0.sum() + 10.0
        sense[-1] = 0
    return A, b, c, sense
