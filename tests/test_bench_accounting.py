"""The benchmark's algorithmic byte count (the roofline's numerator), checked
against a step-by-step enumeration of the filter schedule: which steps read
and write V, and that every coefficient mu_0 .. mu_n enters V exactly once."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def schedule(n):
    """(kappa, coefficients added to V) for steps 1 .. n of a degree-n filter:
    step 1 writes W2 = B V (reads V, writes W2); step 2 forms W1 and sets
    V = mu0 V + mu1 W2 + mu2 W1; from step 3 on, even steps add two terms
    (the previous step's vector and this one's), odd steps run the
    recurrence alone, and an odd last step adds its own term."""
    steps = [(2, []), (4, [0, 1, 2])]
    for k in range(3, n + 1):
        if k % 2 == 0:
            steps.append((5, [k - 1, k]))
        elif k == n:
            steps.append((5, [k]))
        else:
            steps.append((3, []))
    return steps


@pytest.mark.parametrize("n", list(range(2, 30)) + [500, 501, 800])
def test_every_coefficient_once_and_byte_count(n):
    st = schedule(n)
    assert len(st) == n  # exactly n SpMMVs (Alg. 2)
    added = sorted(c for _, cs in st for c in cs)
    assert added == list(range(n + 1))
    n5 = sum(1 for k, (kap, _) in enumerate(st) if k >= 2 and kap == 5)
    n3 = sum(1 for k, (kap, _) in enumerate(st) if k >= 2 and kap == 3)
    assert bench.filter_step_counts(n) == (n5, n3)
    nnz, D, nb, sv = 56_000_000, 8_000_000, 64, 8
    want = sum(nnz * (sv + 4) + 4 * (D + 1) + kap * D * nb * sv for kap, _ in st)
    assert bench.filter_bytes(nnz, D, nb, sv, n) == want


def test_headline_bytes_per_launch():
    """Degree 500, nb = 64, FP64 on Anderson L=200: the per-launch average
    that the roofline reports (17,071,616,004 bytes)."""
    fb = bench.filter_bytes(56_000_000, 8_000_000, 64, 8, 500)
    assert fb / 500 == pytest.approx(17_071_616_004, abs=1)
