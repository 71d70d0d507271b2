"""Pins of the truncation rule (Appendix A.2) and of the reading that
keeps or drops runs of nearly equal singular values whole."""
import numpy as np
import pytest

from oracle import pt_tebd
from oracle.build import problem_from_workload
from oracle.pt_tebd import truncation_rank
from paper_2201_05529_amd import workloads as W


def test_truncation_rule_examples():
    # the smallest rank whose discarded tail has 2-norm strictly below eps
    # times the largest singular value
    sv = np.array([1.0, 1e-3, 1e-8, 1e-9])
    assert truncation_rank(sv, 1e-7) == 2
    assert truncation_rank(sv, 1e-4) == 2
    assert truncation_rank(sv, 1e-2) == 1
    assert truncation_rank(sv, 0.0) == 4
    assert truncation_rank(np.array([1.0, 0.0, 0.0]), 0.0) == 1
    assert truncation_rank(np.array([1.0, 0.5, 0.5, 0.1]), 0.0, chi_max=2) == 1  # run split by the cap
    assert truncation_rank(np.array([1.0, 0.5, 0.4, 0.1]), 0.0, chi_max=2) == 2
    # the tail beyond rank 3 of [1, 1e-3, 9e-8, 9e-8] is 9e-8 < 1e-7 (beyond
    # rank 2 it is 1.3e-7): the minimal rank is 3, which splits the run of
    # two equal values; the run is kept whole
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 9e-8]), 1e-7, tie=0.0) == 3
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 9e-8]), 1e-7) == 4
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 8e-8]), 1e-7) == 3
    # relative gap just above / below 1e-6
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 9e-8 * (1 - 2e-6)]), 1e-7) == 3
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 9e-8 * (1 - 5e-7)]), 1e-7) == 4
    # the cap lowers to the start of a run
    assert truncation_rank(np.array([1.0, 1e-3, 9e-8, 9e-8]), 1e-7, chi_max=3) == 2


def test_truncation_rule_is_the_minimal_admissible_rank():
    # brute force over every candidate rank: without runs (tie = 0) the
    # rule returns the smallest c with ||sv[c:]||_2 < eps sv[0]; with runs,
    # the smallest admissible c that does not split a run
    rng = np.random.default_rng(11)
    for trial in range(400):
        n = int(rng.integers(1, 30))
        sv = np.sort(10.0 ** rng.uniform(-12, 0, size=n))[::-1]
        if trial % 5 == 0:
            sv[n // 2:] = 0.0
        if trial % 3 == 0 and n > 3:  # plant an exact pair
            i = int(rng.integers(1, n - 1))
            sv[i + 1] = sv[i]
        eps = 10.0 ** rng.uniform(-9, -1)
        npos = int(np.count_nonzero(sv > 0))

        def admissible(c):
            return c == npos or np.sqrt(np.sum(sv[c:npos] ** 2)) < eps * sv[0]

        def splits(c):
            return 0 < c < npos and sv[c - 1] - sv[c] < 1e-6 * sv[c - 1]

        want0 = min([c for c in range(1, npos + 1) if admissible(c)]) if npos else 1
        assert truncation_rank(sv, eps, tie=0.0) == want0
        want = min([c for c in range(1, npos + 1) if admissible(c) and not splits(c)]) if npos else 1
        assert truncation_rank(sv, eps) == want
        cap = int(rng.integers(1, n + 1))
        got = truncation_rank(sv, eps, chi_max=cap)
        if want <= cap:
            assert got == want
        else:
            assert 1 <= got <= cap
            assert got == 1 or not splits(got)
            assert all(splits(c) for c in range(got + 1, cap + 1))


@pytest.mark.parametrize("name,steps,bound_runs,gap_plain", [("xyz3", 40, 1e-10, None), ("xyz5", 30, 1e-10, 2e-7)])
def test_runs_make_the_truncated_trajectory_well_defined(name, steps, bound_runs, gap_plain):
    # two LAPACK drivers (divide and conquer, QR iteration) are two correct
    # implementations of every SVD of the method.  With runs kept or dropped
    # whole their trajectories agree to rounding level; with the minimal rank
    # alone they separate on the N = 5 workload, because cuts fall between
    # nearly equal singular values whose kept vectors rounding can exchange
    wl = getattr(W, name)()
    prob, _ = problem_from_workload(wl, n_steps=steps)
    n = wl["n_sites"]

    def run(driver, tie):
        eng = pt_tebd.Engine(prob, svd_driver=driver, tie=tie)
        out = []
        for _ in range(steps):
            eng.step(1)
            out.append([eng.expectation(s, W.SZ) for s in range(n)])
        return np.array(out)

    runs = np.abs(run("gesdd", 1e-6) - run("gesvd", 1e-6)).max()
    print(f"{name}: drivers apart by {runs:.1e} with runs kept whole")
    assert runs < bound_runs
    if gap_plain is not None:
        plain = np.abs(run("gesdd", 0.0) - run("gesvd", 0.0)).max()
        print(f"{name}: drivers apart by {plain:.1e} with the minimal rank alone")
        assert plain > gap_plain
