"""GPU parity: the HIP path, called through the C ABI, reproduces the CPU
oracle bit for bit -- status, pivot sequence, x, objective, duals, basis and
(where requested) the whole tableau -- on both schedules, several grid sizes,
ragged shapes, edge cases and the full-size workloads (sampled)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests import lp_checks
from tests.gpu_util import announce, assert_bitwise_equal, bits, gpu_solve

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
WG, GRID, CD = lpdense.SCHED_WORKGROUP, lpdense.SCHED_GRID, lpdense.SCHED_GRID_CONDENSED
PAIR, CDPAIR = lpdense.SCHED_GRID_PAIRED, lpdense.SCHED_GRID_CONDENSED_PAIRED
GRIDS = pytest.mark.parametrize("schedule", [GRID, CD, PAIR, CDPAIR],
                                ids=["grid", "condensed", "paired", "condensed_paired"])


def _examples():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("schedule", [WG, GRID, CD, PAIR, CDPAIR],
                         ids=["wg", "grid", "condensed", "paired", "condensed_paired"])
@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["id"])
def test_worked_examples(ex, schedule):
    A, b, c = (np.array(ex[k], float) for k in ("A", "b", "c"))
    max_iter = ex.get("max_iter", -1)
    announce(f"worked example {ex['id']} schedule={schedule}")
    g = gpu_solve(A, b, c, max_iter=max_iter, schedule=schedule, want_tableau=True)
    ref = oracle.solve(A, b, c, max_iter=None if max_iter < 0 else max_iter, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)
    assert g.status == ex["status"] and g.trace.tolist() == ex["trace"]


@pytest.mark.parametrize("seed", range(100))
def test_config0_64x64_workgroup(seed):
    """64 x 64 generator instances (the small single-LP workload), default schedule."""
    A, b, c = lpgen.dense_lp(64, 64, seed)
    announce(f"64x64 seed={seed} auto schedule")
    g = gpu_solve(A, b, c, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert ref.status == oracle.OPTIMAL
    assert_bitwise_equal(g, ref, check_tableau=True)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 6000), (3, 1500), (7, 900), (120, 10), (100, 40), (33, 31)])
def test_lds_shapes(m, n):
    """The LDS schedule on shapes that stress its walks: rows longer than the
    workgroup (a thread holds several columns of one row), more rows than a
    wave has lanes, a tableau near the LDS limit, and tiny ones."""
    A, b, c = lpgen.dense_lp(m, n, m + n)
    announce(f"LDS schedule {m}x{n}")
    g = gpu_solve(A, b, c, schedule=WG, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)


@pytest.mark.parametrize("schedule", [WG, GRID, CD, PAIR, CDPAIR],
                         ids=["wg", "grid", "condensed", "paired", "condensed_paired"])
@pytest.mark.parametrize("m,n,lo,hi,bv,cv", [(50, 60, 1, 3, 6.0, 5.0), (64, 64, 1, 2, 4.0, 1.0),
                                             (30, 90, 0, 2, 2.0, 3.0)])
def test_heavy_ties(m, n, lo, hi, bv, cv, schedule):
    """Every reduced cost equal at the start, A of a few small integers (some
    zero) and a constant b: many exact ties in pricing and in the ratio test,
    and degenerate pivots; the lowest index must win each of them."""
    rng = np.random.default_rng(7 + m + n)
    A = rng.integers(lo, hi + 1, size=(m, n)).astype(float)
    b, c = np.full(m, bv), np.full(n, cv)
    announce(f"heavy ties {m}x{n} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert ref.status == oracle.OPTIMAL
    assert_bitwise_equal(g, ref, check_tableau=True)


@GRIDS
@pytest.mark.parametrize("seed", range(20))
def test_config0_64x64_grid(seed, schedule):
    A, b, c = lpgen.dense_lp(64, 64, seed)
    announce(f"64x64 seed={seed} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)


RAGGED = [(1, 1), (1, 9), (9, 1), (2, 3), (3, 300), (300, 3), (33, 65), (129, 257), (257, 129),
          (500, 333), (333, 500), (640, 1281), (1000, 700), (31, 2049)]


@GRIDS
@pytest.mark.parametrize("m,n", RAGGED)
def test_ragged_shapes_grid(m, n, schedule):
    """Shapes spanning several grid-stride sweeps with ragged row / vector tails."""
    A, b, c = lpgen.dense_lp(m, n, 7 + m + n)
    announce(f"ragged {m}x{n} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, want_tableau=m * n <= 400_000)
    ref = oracle.solve(A, b, c, want_tableau=m * n <= 400_000)
    assert_bitwise_equal(g, ref, check_tableau=m * n <= 400_000)


@GRIDS
@pytest.mark.parametrize("m,n,K", [(200, 300, 7), (700, 500, 23), (1025, 1023, 40)])
def test_tableau_after_k_pivots(m, n, K, schedule):
    """max_iter = K stops after K pivots; the whole tableau then matches (the
    condensed schedule rebuilds the full tableau from its nonbasic columns)."""
    A, b, c = lpgen.dense_lp(m, n, 100 + K)
    announce(f"tableau after {K} pivots {m}x{n} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, max_iter=K, want_tableau=True)
    ref = oracle.solve(A, b, c, max_iter=K, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)


@GRIDS
@pytest.mark.parametrize("blocks", [1, 2, 3, 7, 64, 255, 256, 512, 0])
def test_grid_size_invariance(blocks, schedule):
    """Any grid size gives the same bits (a race would show up as a difference);
    sizes past the co-resident limit are clamped to it."""
    A, b, c = lpgen.dense_lp(300, 451, 5)
    announce(f"grid blocks={blocks} 300x451 schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, grid_blocks=blocks, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)


@pytest.mark.parametrize("schedule", [WG, GRID, CD, PAIR, CDPAIR],
                         ids=["wg", "grid", "condensed", "paired", "condensed_paired"])
def test_edge_cases(schedule):
    A = np.array([[1.0, 2.0], [3.0, 1.0]])
    cases = {
        "negative_b": (A, np.array([1.0, -2.0]), np.array([1.0, 1.0])),
        "nan_A": (np.array([[1.0, np.nan], [3.0, 1.0]]), np.array([1.0, 2.0]), np.array([1.0, 1.0])),
        "inf_c": (A, np.array([1.0, 2.0]), np.array([np.inf, 1.0])),
        "unbounded": (np.array([[0.0, 1.0]]), np.array([1.0]), np.array([1.0, 1.0])),
        "already_optimal": (A, np.array([1.0, 2.0]), np.array([-1.0, 0.0])),
        "degenerate_zero_b": (A, np.array([0.0, 0.0]), np.array([1.0, 1.0])),
        # the second pivot of a pair finds no eligible row: one pivot, then UNBOUNDED
        "unbounded_second": (np.array([[1.0, 0.0]]), np.array([1.0]), np.array([2.0, 1.0])),
        # optimal after the first pivot of a pair
        "optimal_after_first": (np.array([[1.0, 1.0]]), np.array([1.0]), np.array([1.0, 0.5])),
    }
    for name, (A_, b_, c_) in cases.items():
        announce(f"edge case {name} schedule={schedule}")
        for max_iter in (-1, 0, 1):
            g = gpu_solve(A_, b_, c_, schedule=schedule, max_iter=max_iter, want_tableau=True)
            ref = oracle.solve(A_, b_, c_, max_iter=None if max_iter < 0 else max_iter, want_tableau=True)
            assert_bitwise_equal(g, ref, check_tableau=name not in ("nan_A", "inf_c"))


def test_workgroup_and_grid_agree_and_errors():
    A, b, c = lpgen.dense_lp(40, 50, 3)
    announce("wg vs grid 40x50")
    g1 = gpu_solve(A, b, c, schedule=WG, want_tableau=True)
    g2 = gpu_solve(A, b, c, schedule=GRID, want_tableau=True)
    g3 = gpu_solve(A, b, c, schedule=CD, want_tableau=True)
    assert np.array_equal(bits(g1.tableau), bits(g2.tableau))
    assert np.array_equal(bits(g1.tableau), bits(g3.tableau))
    import torch
    tA = torch.zeros((400, 400), dtype=torch.float64, device="cuda")
    tb = torch.ones(400, dtype=torch.float64, device="cuda")
    tc = torch.ones(400, dtype=torch.float64, device="cuda")
    with pytest.raises(lpdense.LpdError) as e:  # tableau far beyond LDS
        lpdense.solve_dense_ex(tA, tb, tc, schedule=WG)
    assert e.value.code == -7


@pytest.mark.parametrize("schedule", [lpdense.SCHED_AUTO, CD, PAIR, CDPAIR],
                         ids=["auto", "condensed", "paired", "condensed_paired"])
@pytest.mark.parametrize("m,n,seed", [(1024, 1024, 0), (2048, 512, 1), (512, 2048, 2)])
def test_medium_full_solve(m, n, seed, schedule):
    A, b, c = lpgen.dense_lp(m, n, seed)
    announce(f"medium full solve {m}x{n} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule)
    ref = oracle.solve(A, b, c)
    assert_bitwise_equal(g, ref)
    rp, rd, gap = lp_checks.residuals(A, b, c, g.x, g.y)
    assert rp <= 1e-9 and rd <= 1e-9 and gap <= 1e-9


@pytest.mark.parametrize("schedule", [lpdense.SCHED_AUTO, GRID, CD, PAIR, CDPAIR],
                         ids=["auto", "grid", "condensed", "paired", "condensed_paired"])
@pytest.mark.parametrize("m,n,seed", [(30, 40, 1), (256, 512, 2), (512, 256, 3), (700, 900, 4)])
def test_paper_generator_instances(m, n, seed, schedule):
    """The second workload (zeros in A, b = A x0, c of both signs: many
    pricing ties and degenerate pivots) gives the oracle's bits too."""
    A, b, c = lpgen.paper_lp(m, n, seed)
    announce(f"paper-style {m}x{n} seed={seed} schedule={schedule}")
    small = m * n <= 300_000
    g = gpu_solve(A, b, c, schedule=schedule, want_tableau=small)
    ref = oracle.solve(A, b, c, want_tableau=small)
    assert ref.status == oracle.OPTIMAL
    assert_bitwise_equal(g, ref, check_tableau=small)


@pytest.mark.parametrize("blocks,schedule", [(2, GRID), (3, GRID), (5, GRID), (2, CD), (3, CD), (2, PAIR), (3, PAIR),
                                             (2, CDPAIR), (3, CDPAIR)],
                         ids=["grid2", "grid3", "grid5", "condensed2", "condensed3", "paired2", "paired3",
                              "condensed_paired2", "condensed_paired3"])
def test_dynamic_sweep_bitwise(blocks, schedule):
    """A sweep of at least 48 grid steps hands all but its first 16 steps out
    in chunks through two ticket counters (even and odd chunks); workgroups
    of even and odd rank start on different counters and take from the other
    once theirs runs dry.  On a grid of a few workgroups a 700 x 1000 LP is
    long enough for that; a chunk lost, done twice or taken from the wrong
    pivot's counter would change bits, so the whole tableau must match the
    oracle."""
    m, n = 700, 1000
    vw = (n + 1) // 2 if schedule == CD else (n + m + 1) // 2
    assert -(-m * vw // (blocks * 1024)) >= 48  # long enough for the ticket path
    A, b, c = lpgen.dense_lp(m, n, 11)
    announce(f"dynamic sweep {m}x{n} blocks={blocks} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, grid_blocks=blocks, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert ref.status == oracle.OPTIMAL
    assert_bitwise_equal(g, ref, check_tableau=True)


@GRIDS
@pytest.mark.parametrize("m,n,seed", [(120, 90, 7), (300, 400, 8)])
def test_one_workgroup_team(m, n, seed, schedule):
    """A grid of one workgroup: the team barriers, and the pair's counter
    barrier on the paired schedules, reduce to workgroup barriers."""
    A, b, c = lpgen.dense_lp(m, n, seed)
    announce(f"one-workgroup team {m}x{n} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, grid_blocks=1, want_tableau=True)
    ref = oracle.solve(A, b, c, want_tableau=True)
    assert_bitwise_equal(g, ref, check_tableau=True)


PAIRS = pytest.mark.parametrize("schedule", [PAIR, CDPAIR], ids=["paired", "condensed_paired"])


@PAIRS
@pytest.mark.parametrize("max_iter", [2, 3, 4, 5, 7])
def test_pair_iteration_caps(max_iter, schedule):
    """An odd cap ends on a sweep of one pivot; the tableau at the cap is the
    oracle's either way."""
    A, b, c = lpgen.dense_lp(200, 300, 9)
    announce(f"pair iteration cap {max_iter} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, max_iter=max_iter, want_tableau=True)
    ref = oracle.solve(A, b, c, max_iter=max_iter, want_tableau=True)
    assert ref.status == oracle.ITERATION_LIMIT
    assert_bitwise_equal(g, ref, check_tableau=True)


@PAIRS
@pytest.mark.parametrize("cap", [1, 4, 5])
def test_pair_trace_capacity(cap, schedule):
    """A trace shorter than the solve keeps its first `cap` pivots, also when
    the capacity ends between the two pivots of a sweep."""
    A, b, c = lpgen.dense_lp(200, 300, 9)
    announce(f"pair trace capacity {cap} schedule={schedule}")
    g = gpu_solve(A, b, c, schedule=schedule, trace_cap=cap)
    ref = oracle.solve(A, b, c)
    assert g.iterations == ref.iterations > cap
    assert np.array_equal(g.trace, ref.trace[:cap])
    assert np.array_equal(bits(g.x), bits(ref.x))
