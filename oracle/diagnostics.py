"""Neighbour-triggered flip rate P_NT(t) of a recorded trajectory
(Suppl. "Quantifying coupled oscillatory dynamics via neighbor-triggered flip
rates", definition of P_NT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` do.

For each spin i of each trial at step t: spin i has a flipping neighbour when
some j with J_ij != 0 flips between s(t) and s(t+1); P_NT(t) is the
probability that i itself flips given that, averaged over spins and trials.
Reading where the paper is silent: the average is the pooled ratio
    P_NT(t) = #{(i, a): i flips and a neighbour flips} / #{(i, a): a neighbour flips},
undefined (NaN) when no spin of any trial has a flipping neighbour.
"""
import numpy as np


def neighbor_flip_counts(J, states):
    """states: int [T + 1, N, R] (s(t) at index t).  Returns (num, den), int64
    arrays of length T, written out with explicit loops over the definition."""
    J = np.asarray(J)
    adj = (J != 0)
    np.fill_diagonal(adj, False)
    states = np.asarray(states)
    T = states.shape[0] - 1
    n, R = states.shape[1], states.shape[2]
    num = np.zeros(T, dtype=np.int64)
    den = np.zeros(T, dtype=np.int64)
    for t in range(T):
        flipped = states[t + 1] != states[t]  # [N, R]
        # neighbour_flips[i, a] = number of neighbours j of i that flip in trial a
        neighbour_flips = adj.astype(np.int64) @ flipped.astype(np.int64)
        has = neighbour_flips > 0
        den[t] = int(has.sum())
        num[t] = int((has & flipped).sum())
    return num, den


def neighbor_flip_rate(J, states):
    num, den = neighbor_flip_counts(J, states)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(den > 0, num / np.maximum(den, 1), np.nan)
