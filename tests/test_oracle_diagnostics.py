"""Pins for the neighbour-triggered flip rate (oracle/diagnostics.py)."""
import numpy as np

import workloads as w
from oracle import diagnostics, pimi


def _brute(J, states):
    """Literal per-(t, i, a) loops over the definition."""
    T1, n, R = states.shape
    num = np.zeros(T1 - 1, np.int64)
    den = np.zeros(T1 - 1, np.int64)
    for t in range(T1 - 1):
        for a in range(R):
            for i in range(n):
                nb = any(J[i][j] != 0 and j != i and states[t + 1, j, a] != states[t, j, a] for j in range(n))
                if nb:
                    den[t] += 1
                    num[t] += int(states[t + 1, i, a] != states[t, i, a])
    return num, den


def test_counts_match_literal_loops():
    rng = np.random.default_rng(5)
    J, _ = w.random_int8(7, seed=1, index=0, jmax=1, density=0.4)
    states = rng.choice([-1, 1], size=(9, 7, 3)).astype(np.int8)
    num, den = diagnostics.neighbor_flip_counts(J, states)
    bn, bd = _brute(J, states)
    assert np.array_equal(num, bn) and np.array_equal(den, bd)


def test_complete_graph_closed_form():
    """On a complete graph with m flips in a trial: num = m [m >= 2] and
    den = N [m >= 2] + (N - 1) [m == 1]."""
    n = 6
    J = np.ones((n, n), np.int64) - np.eye(n, dtype=np.int64)
    base = np.ones(n, np.int8)
    for m in range(n + 1):
        nxt = base.copy()
        nxt[:m] = -1
        states = np.stack([base, nxt])[:, :, None]
        num, den = diagnostics.neighbor_flip_counts(J, states)
        assert num[0] == (m if m >= 2 else 0)
        assert den[0] == (n if m >= 2 else (n - 1 if m == 1 else 0))


def test_no_edges_is_undefined_and_frozen_is_zero_numerator():
    states = np.ones((4, 5, 2), np.int8)
    states[2, 0, 0] = -1
    assert np.all(np.isnan(diagnostics.neighbor_flip_rate(np.zeros((5, 5)), states)))
    J = np.ones((5, 5)) - np.eye(5)
    num, den = diagnostics.neighbor_flip_counts(J, np.ones((4, 5, 2), np.int8))
    assert not num.any() and not den.any()


def test_inertia_suppresses_neighbour_triggered_flips():
    """The paper's trend (qualitative, pin P8): late-anneal P_NT falls as xi
    grows; high without inertia (about 0.6 with the 4-level LUT and this
    schedule), near zero at xi = 1."""
    n, R, T = 32, 64, 160
    J, h = w.sk1(n, seed=3, index=0)
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    late = []
    for xi in (0.0, 0.5, 1.0):
        prob = pimi.Problem(J, h, 1 / np.sqrt(n), xi, 4, w.gauss_table(8))
        res = pimi.run_parallel(prob, beta, eta, 4, 0, np.arange(R), record=True)
        p = diagnostics.neighbor_flip_rate(J, res["states"])
        late.append(float(np.nanmean(p[T // 2:])) if np.any(np.isfinite(p[T // 2:])) else 0.0)
    assert late[0] > 0.4 and late[0] > 4 * late[1] and late[1] > late[2] and late[2] < 0.05, late
