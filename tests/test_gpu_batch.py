"""Batched solve (lp_solve_batch): every LP of a batch gets exactly the bits
its own single solve and the CPU oracle give, whatever the batch composition,
order, team size or class threshold."""
import hashlib
import os

import numpy as np
import pytest

import oracle
from paper_1804_04737_amd import lpdense, lpgen
from tests import lp_checks
from tests.gpu_util import announce, bits

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _run_batch(lps, **kw):
    import torch
    pb = lpdense.pack_batch(lps)
    lpdense.solve_batch(pb, **kw)
    torch.cuda.synchronize()
    return ([pb.x_of(i).cpu().numpy() for i in range(pb.count)], pb.obj.cpu().numpy(),
            pb.status.cpu().numpy(), pb.iterations.cpu().numpy())


def _mixed_lps(seed, count=40):
    """Shapes chosen to hit all three classes: LDS-resident, one workgroup in
    HBM, and team-solved (with a low team threshold)."""
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(1, 40)), int(rng.integers(1, 40))) for _ in range(count // 2)]
    shapes += [(int(rng.integers(60, 400)), int(rng.integers(60, 500))) for _ in range(count // 2 - 4)]
    shapes += [(700, 900), (1024, 300), (257, 1500), (900, 1024)]
    return [lpgen.dense_lp(m, n, 1000 * seed + i) for i, (m, n) in enumerate(shapes)]


@pytest.mark.parametrize("full", [False, True], ids=["condensed", "full"])
@pytest.mark.parametrize("team_size,team_min", [(0, 0), (1, 0), (2, 200_000), (8, 200_000), (32, 1_000_000)])
def test_batch_equals_oracle(team_size, team_min, full):
    lps = _mixed_lps(1)
    announce(f"batch of {len(lps)} team_size={team_size} team_min={team_min} full_tableau={full}")
    xs, obj, st, it = _run_batch(lps, team_size=team_size, team_min_bytes=team_min, full_tableau=full)
    for i, (A, b, c) in enumerate(lps):
        ref = oracle.solve(A, b, c)
        assert st[i] == ref.status and it[i] == ref.iterations, i
        assert np.array_equal(bits(xs[i]), bits(ref.x)), i
        assert bits([obj[i]])[0] == bits([ref.obj])[0], i


def test_batch_order_and_single_solve_agree():
    import torch
    lps = _mixed_lps(2, count=24)
    announce("batch order invariance")
    xs1, obj1, st1, it1 = _run_batch(lps, team_size=4, team_min_bytes=300_000)
    perm = np.random.default_rng(5).permutation(len(lps))
    xs2, obj2, st2, it2 = _run_batch([lps[p] for p in perm], team_size=16, team_min_bytes=100_000,
                                     full_tableau=True)
    dev = torch.device("cuda")
    for j, p in enumerate(perm):
        assert np.array_equal(bits(xs1[p]), bits(xs2[j])) and bits([obj1[p]])[0] == bits([obj2[j]])[0]
        assert st1[p] == st2[j] and it1[p] == it2[j]
        A, b, c = lps[p]
        r = lpdense.solve_dense_ex(*(torch.from_numpy(v).to(dev) for v in (A, b, c)))
        torch.cuda.synchronize()
        assert np.array_equal(bits(r.x.cpu().numpy()), bits(xs1[p]))
        assert int(r.status.item()) == st1[p]


def _tiny_lps(seed, count=60):
    """Mostly tiny LPs (one wave each when wave slots are on) plus a few
    larger ones for the other classes."""
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(1, 30)), int(rng.integers(1, 30))) for _ in range(count - 6)]
    shapes += [(45, 50), (60, 40), (120, 90), (300, 200), (1, 200), (200, 1)]
    return [lpgen.dense_lp(m, n, 5000 * seed + i) for i, (m, n) in enumerate(shapes)]


@pytest.mark.parametrize("wave_slots", [2, 4, 16])
def test_batch_wave_per_instance_equals_oracle(wave_slots):
    """One wave per tiny LP (its tableau in the wave's LDS slice): bits equal
    the oracle's, and equal the same batch solved with wave slots off."""
    lps = _tiny_lps(wave_slots)
    announce(f"batch wave_slots={wave_slots}, {len(lps)} LPs")
    xs, obj, st, it = _run_batch(lps, wave_slots=wave_slots)
    xs0, obj0, st0, it0 = _run_batch(lps, wave_slots=-1)
    for i, (A, b, c) in enumerate(lps):
        ref = oracle.solve(A, b, c)
        assert st[i] == ref.status and it[i] == ref.iterations, i
        assert np.array_equal(bits(xs[i]), bits(ref.x)), i
        assert bits([obj[i]])[0] == bits([ref.obj])[0], i
        assert np.array_equal(bits(xs[i]), bits(xs0[i])) and it[i] == it0[i]


@pytest.mark.parametrize("wave_slots", [-1, 8])
def test_batch_with_edge_cases(wave_slots):
    A = np.array([[1.0, 2.0], [3.0, 1.0]])
    lps = [
        (A, np.array([1.0, -2.0]), np.array([1.0, 1.0])),                          # INFEASIBLE_START
        (np.array([[1.0, np.nan], [3.0, 1.0]]), np.array([1.0, 2.0]), np.ones(2)),  # NUMERICAL
        (np.array([[0.0, 1.0]]), np.array([1.0]), np.array([1.0, 1.0])),          # UNBOUNDED
        (A, np.array([1.0, 2.0]), np.array([-1.0, 0.0])),                          # already optimal
        lpgen.dense_lp(300, 200, 3),
        (np.array([[0.0, 1.0]]), np.array([1.0]), np.array([1.0, 1.0])),
        lpgen.dense_lp(500, 600, 4),
    ]
    announce(f"batch edge cases wave_slots={wave_slots}")
    xs, obj, st, it = _run_batch(lps, team_size=4, team_min_bytes=1_000_000, wave_slots=wave_slots)
    for i, (A_, b_, c_) in enumerate(lps):
        ref = oracle.solve(A_, b_, c_)
        assert st[i] == ref.status and it[i] == ref.iterations
        assert np.array_equal(bits(xs[i]), bits(ref.x))


@pytest.mark.parametrize("full", [False, True], ids=["condensed", "full"])
def test_batch_with_rows_longer_than_lds(full):
    """The batch kernel walks each LP with its pivot row in LDS.  LPs whose
    row does not fit (10 x 25000, 6 x 40000) are solved after the batch on
    the grid schedule with two pivots per sweep and column panels; every
    result, theirs included, equals the oracle's bits."""
    lps = [lpgen.dense_lp(20, 30, 1), lpgen.dense_lp(10, 25000, 2), lpgen.dense_lp(300, 200, 3),
           lpgen.dense_lp(6, 40000, 4), lpgen.dense_lp(64, 64, 5)]
    announce(f"batch with rows longer than the LDS full_tableau={full}")
    xs, obj, st, it = _run_batch(lps, full_tableau=full)
    for i, (A, b, c) in enumerate(lps):
        ref = oracle.solve(A, b, c)
        assert st[i] == ref.status and it[i] == ref.iterations, (i, st[i], ref.status)
        assert np.array_equal(bits(xs[i]), bits(ref.x)), i
        assert bits([obj[i]])[0] == bits([ref.obj])[0], i


def test_batch_max_iter_applies_to_each_lp():
    lps = _mixed_lps(3, count=12) + _tiny_lps(3, count=12)
    announce("batch max_iter=5")
    xs, obj, st, it = _run_batch(lps, max_iter=5, wave_slots=4)
    for i, (A, b, c) in enumerate(lps):
        ref = oracle.solve(A, b, c, max_iter=5)
        assert st[i] == ref.status and it[i] == ref.iterations
        assert np.array_equal(bits(xs[i]), bits(ref.x))


def test_batched_workload_1024():
    """The batched workload: 1024 LPs, m and n log-uniform in [32, 1024],
    default (autotuned) schedule.  Every LP equals the oracle's solve of it:
    status, pivot count, the bits of z and the SHA-256 of the bits of x
    (stored in tests/golden/batch1024_seed0.npz by
    tests/golden/make_oracle_goldens.py, which runs only the CPU oracle); and
    every x is feasible with c^T x = z within 1e-9."""
    lps = lpgen.batch_lps(1024, 32, 1024, 0)
    with np.load(os.path.join(GOLDEN, "batch1024_seed0.npz"), allow_pickle=False) as z:
        ref = {k: z[k] for k in z.files}
    assert int(ref["count"]) == 1024 and (int(ref["lo"]), int(ref["hi"]), int(ref["seed"])) == (32, 1024, 0)
    announce("batched workload 1024 LPs")
    xs, obj, st, it = _run_batch(lps)
    assert np.array_equal(st, ref["status"])
    assert np.array_equal(it, ref["iterations"])
    assert np.array_equal(bits(obj), ref["obj_bits"])
    bad = [i for i in range(1024)
           if hashlib.sha256(np.ascontiguousarray(xs[i], dtype="<f8").tobytes()).digest() != ref["x_sha256"][i].tobytes()]
    assert not bad, f"x differs from the oracle's for LPs {bad[:10]}"
    for i, (A, b, c) in enumerate(lps):
        assert abs(float(c @ xs[i]) - obj[i]) <= 1e-9 * max(1.0, abs(obj[i]))
        assert float(np.max(A @ xs[i] - b)) <= 1e-9 * (1 + float(np.max(b)))
        assert float(np.min(xs[i])) >= 0.0
