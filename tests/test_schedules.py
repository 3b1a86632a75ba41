"""Host-side schedules of the library (paper_2506_04976_amd.schedules) against
the oracle's independently written rules, and the per-epoch plans of ALG1,
ALG2 and ALG3 (Section 4 and its table of hyperparameters)."""

import numpy as np
import pytest

from oracle import recon
from oracle import schedules as orc
from paper_2506_04976_amd import schedules as lib


@pytest.mark.parametrize("n", list(range(1, 65)))
def test_orders_match_oracle(n):
    assert lib.herman_meyer_order(n) == orc.herman_meyer(n)
    assert lib.cofactor_order(n, 9) == orc.cofactor_orders(n, 9)


def test_subset_count_matches_oracle():
    for views in range(1, 520):
        for target in (25.0, 24.2):
            assert lib.subsets_for(views, target) == orc.n_subsets_closest(views, target)


def test_stepsizes_match_oracle():
    for k in range(0, 400):
        assert lib.alg1_tau(k) == recon.stepsize_alg1(k)
        for n in (8, 21, 25, 28):
            assert lib.alg23_cap(k, n) == orc.alg2_cap(k, n)


@pytest.mark.parametrize("alg", ["ALG1", "ALG2", "ALG3"])
def test_algorithm_plans(alg):
    n, E = 21, 8
    plan = lib.algorithm_plan(alg, n, E, np.random.default_rng(3))
    assert len(plan) == E
    pc = [e * n + j for e in range(E) for j in range(n) if plan[e]["update_pc"][j]]
    assert pc == ([0, n, 2 * n] if alg == "ALG1" else [0, n, 3 * n, 5 * n])
    for e, p in enumerate(plan):
        assert sorted(p["subset_seq"]) == list(range(n))
        if alg == "ALG3":
            assert p["subset_seq"] == orc.cofactor_orders(n, E)[e]
    if alg == "ALG1":
        assert all(p["bb_update"] is None for p in plan)
        assert plan[0]["tau"][0] == 3.0 and plan[E - 1]["tau"][-1] == recon.stepsize_alg1(E * n - 1)
    else:
        bb = [e * n + j for e in range(E) for j in range(n) if plan[e]["bb_update"][j]]
        assert bb == [2 * n, 4 * n, 6 * n]
        # BB updates fall on snapshot iterations (omega = 2)
        assert all(k % (2 * n) == 0 for k in bb)
    with pytest.raises(ValueError):
        lib.algorithm_plan("ALG4", n, 1)
