"""Serving runtime (lpd_server_*): continuous batching with admission by
footprint.  Every result is bit-identical to the oracle's (and so to a solve
of the LP alone) whatever else is resident, however often its solve is
suspended and resumed, and admission never exceeds the budget."""
import time

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu


def _drain(srv, n_expected, timeout=120.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < n_expected:
        for r in srv.poll():
            got[r.id] = r
        if time.time() > t_end:
            raise AssertionError(f"only {len(got)} of {n_expected} requests finished")
        time.sleep(0.001)
    return got


def _check_vs_oracle(lp, r, **kw):
    A, b, c = lp
    ref = oracle.solve(A, b, c, **kw)
    assert r.status == ref.status and r.iterations == ref.iterations, (r.status, ref.status)
    assert np.array_equal(bits(r.x), bits(ref.x))
    assert bits([r.obj])[0] == bits([ref.obj])[0]


def _mix(seed, count):
    rng = np.random.default_rng(seed)
    shapes = []
    for q in range(count):
        if q % 3 == 0:
            shapes.append((int(rng.integers(2, 40)), int(rng.integers(2, 40))))   # LDS-resident
        else:
            shapes.append((int(rng.integers(80, 420)), int(rng.integers(80, 520))))
    return [lpgen.dense_lp(m, n, 7000 + 100 * seed + i) for i, (m, n) in enumerate(shapes)]


@pytest.mark.parametrize("ppe,full", [(1, False), (7, False), (0, False), (3, True)])
def test_server_results_equal_oracle(ppe, full):
    """Teams of several sizes (low thresholds) and a small pivot budget per
    epoch: each LP is suspended and resumed many times, by teams whose size
    changes with the resident mix; condensed and full tableaux."""
    lps = _mix(1, 24)
    announce(f"server mix of {len(lps)} pivots_per_epoch={ppe} full_tableau={full}")
    with lpdense.Server(8 << 30, pivots_per_epoch=ppe, team_min_bytes=150_000,
                        team_bytes_per_wg=60_000, full_tableau=full) as srv:
        ids = [srv.submit(*lp) for lp in lps]
        got = _drain(srv, len(ids))
        st = srv.stats()
        assert st.completed == len(lps) and st.used_bytes == 0
    for i, lp in zip(ids, lps):
        _check_vs_oracle(lp, got[i])


def test_server_arrivals_while_running():
    """Requests that arrive while others are on the device are admitted and
    finish in the same run: a large LP first, small ones during its solve.
    The small ones finish before the large one does."""
    big = lpgen.dense_lp(2500, 2500, 11)
    small = _mix(2, 12)
    announce("server arrivals while a 2500x2500 LP runs")
    with lpdense.Server(8 << 30, pivots_per_epoch=16) as srv:
        bid = srv.submit(*big)
        t0 = time.time()
        while srv.stats().epochs < 2 and time.time() - t0 < 30:
            time.sleep(0.0005)
        sids = [srv.submit(*lp) for lp in small]
        got = _drain(srv, 1 + len(sids))
        st = srv.stats()
    assert st.epochs > 2
    assert max(got[i].t_done for i in sids) < got[bid].t_done
    assert min(got[i].t_admit for i in sids) < got[bid].t_done
    for i, lp in zip(sids, small):
        _check_vs_oracle(lp, got[i])
    A, b, c = big
    x = got[bid].x
    assert got[bid].status == lpdense.OPTIMAL
    assert float(np.max(A @ x - b)) <= 1e-9 * float(np.max(b)) and float(np.min(x)) >= 0.0
    assert abs(float(c @ x) - got[bid].obj) <= 1e-9 * abs(got[bid].obj)


def test_server_admission_respects_budget():
    """A budget that holds about two of the LPs at a time: every LP still
    finishes with the oracle's bits and the resident footprint never exceeds
    the budget."""
    lps = [lpgen.dense_lp(300 + 10 * i, 320, 900 + i) for i in range(8)]
    foot = max(8 * (m * n + m + 2 * n) + 8 * m * (n + m + 64) + 8 * 4 * (n + m + 64) + 64 * 1024
               for m, n in (lp[0].shape for lp in lps))
    budget = int(2.2 * foot)
    announce(f"server budget {budget} bytes")
    with lpdense.Server(budget, pivots_per_epoch=5) as srv:
        ids = [srv.submit(*lp) for lp in lps]
        got = _drain(srv, len(ids))
        st = srv.stats()
    assert 0 < st.peak_bytes <= budget
    assert st.used_bytes == 0
    for i, lp in zip(ids, lps):
        _check_vs_oracle(lp, got[i])
    # Admission in arrival order: admit times are non-decreasing.
    adm = [got[i].t_admit for i in ids]
    assert adm == sorted(adm)


def test_server_rejects_and_edge_cases():
    announce("server edge cases")
    A = np.array([[1.0, 2.0], [3.0, 1.0]])
    lps = [
        (A, np.array([1.0, -2.0]), np.array([1.0, 1.0])),                          # INFEASIBLE_START
        (np.array([[1.0, np.nan], [3.0, 1.0]]), np.array([1.0, 2.0]), np.ones(2)),  # NUMERICAL
        (np.array([[0.0, 1.0]]), np.array([1.0]), np.array([1.0, 1.0])),          # UNBOUNDED
        (A, np.array([1.0, 2.0]), np.array([-1.0, 0.0])),                          # already optimal
        lpgen.dense_lp(300, 200, 3),
        (np.zeros((200, 300)), np.ones(200), np.ones(300)),                        # UNBOUNDED, HBM class
    ]
    with lpdense.Server(1 << 20) as tiny:
        with pytest.raises(lpdense.LpdError) as e:
            tiny.submit(*lpgen.dense_lp(400, 500, 1))   # footprint above the whole budget
        assert e.value.code == -7
    with lpdense.Server(1 << 30, pivots_per_epoch=4, max_iter=7) as srv:
        ids = [srv.submit(*lp) for lp in lps]
        got = _drain(srv, len(ids))
    for i, lp in zip(ids, lps):
        _check_vs_oracle(lp, got[i], max_iter=7)


def test_server_lp_moves_from_one_workgroup_to_a_team():
    """A 640 x 700 LP that shares the device with four 4000 x 4000 LPs runs
    on a single workgroup (its share of the workgroups is below two); once
    they have left, the same LP continues on a team of two whose sweeps are
    long enough for the dynamic tail (ticket counters).  The large LPs
    (c = e_0) are optimal after one pivot, and one pivot per epoch makes the
    hand-over happen after the first epochs.  Every result must equal the
    oracle's bits."""
    bigs = []
    for q in range(4):
        A, b, _ = lpgen.dense_lp(4000, 4000, 30 + q)
        c = np.zeros(4000)
        c[0] = 1.0
        bigs.append((A, b, c))
    small = lpgen.dense_lp(640, 700, 22)
    announce("server: single workgroup then team of two")
    with lpdense.Server(16 << 30, pivots_per_epoch=1, team_min_bytes=1,
                        team_bytes_per_wg=3_000_000) as srv:
        bids = [srv.submit(*lp) for lp in bigs]
        sid = srv.submit(*small)
        got = _drain(srv, 5)
    for i, lp in zip(bids, bigs):
        _check_vs_oracle(lp, got[i])
    _check_vs_oracle(small, got[sid])


@pytest.mark.parametrize("full", [False, True], ids=["condensed", "full"])
def test_server_wide_lps(full):
    """LPs whose pivot row is longer than the LDS (10 x 25000, 6 x 40000)
    run as grid launches of their own each epoch (column panels) beside the
    batched ones; a budget of 3 pivots per epoch makes them suspend and
    resume many times.  Every result equals the oracle's bits."""
    lps = [lpgen.dense_lp(10, 25000, 2), lpgen.dense_lp(300, 200, 3), lpgen.dense_lp(6, 40000, 4),
           lpgen.dense_lp(20, 30, 1), lpgen.dense_lp(700, 900, 5)]
    announce(f"server with wide LPs full_tableau={full}")
    with lpdense.Server(1 << 32, pivots_per_epoch=3, full_tableau=full) as srv:
        ids = [srv.submit(*lp) for lp in lps]
        got = _drain(srv, len(ids))
    for i, lp in zip(ids, lps):
        _check_vs_oracle(lp, got[i])
