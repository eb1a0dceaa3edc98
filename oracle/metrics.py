"""Success probability, trials-to-solution and time-to-solution.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. III.A (Eqs. (5)-(6)) and Suppl. "Estimation of optimal clock
cycles to solution":

* a trial succeeds within T steps if min_{t <= T} H(t) <= theta, with
  theta = f * H_gs (f = 0.999: a relaxed criterion, since H_gs < 0);
* p_j(T) is the fraction of successful trials on instance j, p_bar(T) the mean
  over instances;
* n_trials(T) = ceil(log(eps) / log(1 - p_bar(T))) (Eq. (5)), with eps = 0.001
  in the paper and 0.01 for TTS99;
* the cost of a run is n_trials(T) * T * C_step (Eq. (6)); minimised over T.
"""
import math

import numpy as np


def success_threshold(e_gs, frac=0.999):
    return frac * e_gs


def success_flags(first_hit, steps):
    """X_ij(T): trial reached the threshold at some step t <= T.  ``first_hit``
    is the first step with E(t) <= theta, or -1 if never."""
    first_hit = np.asarray(first_hit)
    return (first_hit >= 0) & (first_hit <= steps)


def success_probability(first_hit, steps):
    return float(success_flags(first_hit, steps).mean())


def n_trials(p_bar, eps=0.001):
    """Eq. (5): ceil(log eps / log(1 - p_bar)); 1 when p_bar = 1, inf when 0."""
    if p_bar >= 1.0:
        return 1
    if p_bar <= 0.0:
        return math.inf
    return int(math.ceil(math.log(eps) / math.log(1.0 - p_bar)))


def cost_to_solution(p_bar, steps, cost_per_step, eps=0.001):
    """Eq. (6): n_trials(T) * T * C_step."""
    n = n_trials(p_bar, eps)
    return n * steps * cost_per_step if n != math.inf else math.inf


def optimal_cost(first_hits, step_grid, cost_per_step, eps=0.001):
    """Minimum over T in ``step_grid`` of Eq. (6), with p_bar(T) the mean over
    instances of the per-instance success fraction.  ``first_hits`` is a list
    of per-instance arrays.  Returns (best cost, best T)."""
    best = (math.inf, None)
    for T in step_grid:
        p_bar = float(np.mean([success_probability(fh, T) for fh in first_hits]))
        c = cost_to_solution(p_bar, T, cost_per_step, eps)
        if c < best[0]:
            best = (c, T)
    return best
