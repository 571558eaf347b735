"""The parity instances exercise the special cases of two pivots per sweep.

The paired schedules take pivots 2j and 2j+1 in one sweep.  Two cases take
their own code paths there: the pair's second pivot row equals its first
(l1 = l: row l after the first pivot is the normalised row itself), and a
pair's first pivot row equals the previous sweep's last one (that row is read
from the kept normalised row, not from the tableau).  The GPU parity tests
compare the paired schedules with the oracle bit for bit on the 64 x 64
generator instances (seeds 0..19) and the paper-style instances; this checks,
from the oracle's pivot sequences alone, that those instances contain both
cases, so the bitwise comparison covers them.
"""
import oracle
from paper_1804_04737_amd import lpgen


def _pair_cases(trace):
    same_row = after_kept = 0
    for j in range(0, len(trace) - 1, 2):
        l0, l1 = trace[j][1], trace[j + 1][1]
        same_row += int(l1 == l0)
        after_kept += int(j > 0 and l0 == trace[j - 1][1])
    return same_row, after_kept


def test_64x64_instances_cover_pair_special_cases():
    same_row = after_kept = 0
    for seed in range(20):
        A, b, c = lpgen.dense_lp(64, 64, seed)
        s, k = _pair_cases(oracle.solve(A, b, c).trace)
        same_row += s
        after_kept += k
    assert same_row > 0 and after_kept > 0, (same_row, after_kept)


def test_paper_style_instance_covers_pair_special_cases():
    A, b, c = lpgen.paper_lp(512, 256, 3)
    s, k = _pair_cases(oracle.solve(A, b, c).trace)
    assert s > 0 and k > 0, (s, k)
