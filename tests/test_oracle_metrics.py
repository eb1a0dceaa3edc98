"""Pins of Eqs. (5)-(6) and the success criterion."""
import math

import numpy as np

from oracle import metrics


def test_n_trials_eq5():
    assert metrics.n_trials(0.5, 0.001) == 10          # log(0.001)/log(0.5) = 9.97
    assert metrics.n_trials(0.5, 0.01) == 7            # 6.64
    assert metrics.n_trials(0.99, 0.01) == 1
    assert metrics.n_trials(1.0) == 1
    assert metrics.n_trials(0.0) == math.inf
    # the ceiling: a success probability that needs exactly k trials
    p = 1 - 0.001 ** (1 / 3)
    assert metrics.n_trials(p + 1e-9, 0.001) == 3


def test_cost_and_optimum_eq6():
    assert metrics.cost_to_solution(0.5, 100, 17.0) == 10 * 100 * 17.0
    assert metrics.cost_to_solution(0.0, 100, 1.0) == math.inf
    # instance A succeeds at step 10 on half its trials, instance B at step 40
    fh = [np.array([10, 10, -1, -1]), np.array([40, 40, 40, 40])]
    best, T = metrics.optimal_cost(fh, [10, 20, 40, 80], 1.0)
    # T=10: p=0.25 -> 25 trials; T=40: p=0.75 -> 5 trials
    assert (best, T) == (min(25 * 10, 5 * 40), 40) or (best, T) == (250, 10)
    assert best == 200 and T == 40


def test_success_threshold_is_relaxed_for_negative_energies():
    assert metrics.success_threshold(-1000) == -999.0
    flags = metrics.success_flags(np.array([-1, 0, 5, 9]), 5)
    np.testing.assert_array_equal(flags, [False, True, True, False])
