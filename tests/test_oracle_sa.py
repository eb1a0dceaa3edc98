"""Pins of the simulated-annealing reference (Suppl. "SK-1 instance
generation", "Ground-truth computation").

The anneal is a heuristic, so it is pinned by what fixes its answer from
outside: exact ground states by enumeration (N <= 20), closed-form ground
states of complete graphs, the Boltzmann law that fixed-temperature Metropolis
must sample, the schedule's printed constants, and the generator it draws from
(equal to the oracle's Philox, which is itself pinned against rocRAND).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as w
from oracle import ground, philox, pimi, sa

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_generator_is_philox4x32_10():
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        want = [int(v) for v in philox.philox4x32_10(*ctr, *key)]
        assert sa.philox(ctr, key).tolist() == want


def test_schedule_constants():
    # T_k = 5 * 0.995^k >= 0.01  <=>  k <= log(0.002) / log(0.995) = 1239.8
    assert sa.count_temperatures(5.0, 0.01, 0.995) == math.floor(math.log(0.01 / 5.0) / math.log(0.995)) + 1 == 1240
    assert sa.count_temperatures(1.0, 0.5, 0.5) == 2
    # the printed per-temperature budgets
    for n in (10, 20, 60):
        assert sa.flips_per_temperature(n) == 10 * n
    for n in (70, 80, 90, 100):
        assert sa.flips_per_temperature(n) == 10_000
    for n in (110, 120, 130, 140, 150):
        assert sa.flips_per_temperature(n) == 20_000
    assert sa.flips_per_temperature(200) == 50_000


def test_reaches_enumerated_ground_states_sk20():
    rows = json.load(open(os.path.join(GOLDEN, "sk20_ground_all.json")))
    for row in rows:
        J, h = w.sk1(20, seed=row["seed"], index=row["index"])
        e, s, per_run = sa.anneal(J, h, 1 / math.sqrt(20), seed=3, stream=row["index"])
        assert e == row["e_gs"]
        assert pimi.energy(J, h, s.astype(np.int64)) == e
        assert per_run.min() == e and per_run.shape == (10,)


@pytest.mark.parametrize("index", range(4))
def test_reaches_enumerated_ground_states_with_fields(index):
    J, h = w.random_int8(14, seed=11, index=index, jmax=9, hmax=12)
    e_gs, _, _ = ground.brute_force(J, h)
    e, s, _ = sa.anneal(J, h, 0.1, seed=2, stream=index)
    assert e == e_gs
    assert pimi.energy(J, h, s.astype(np.int64)) == e


@pytest.mark.parametrize("n", [199, 200])
def test_complete_graph_closed_forms(n):
    ones = np.ones((n, n), dtype=np.int8) - np.eye(n, dtype=np.int8)
    zero = np.zeros(n, dtype=np.int32)
    c = 1 / math.sqrt(n)
    # ferromagnet: all spins aligned, E = -N(N-1)/2
    e, s, _ = sa.anneal(ones, zero, c, runs=1, flips=2 * n)
    assert e == -n * (n - 1) // 2 and abs(int(s.astype(np.int64).sum())) == n
    # antiferromagnet J = -1: E = (M^2 - N) / 2 with M = sum s, least at |M| = N mod 2
    e, s, _ = sa.anneal(-ones, zero, c, runs=1, flips=2 * n)
    assert e == ((n % 2) - n) // 2 and abs(int(s.astype(np.int64).sum())) == n % 2


def test_metropolis_samples_boltzmann():
    """Fixed-temperature Metropolis has the Boltzmann law exp(-c E / T) / Z as
    its stationary distribution (detailed balance); a wrong sign of dE, a lost
    c or an inverted acceptance would move it far away."""
    n = 6
    J, h = w.random_int8(n, seed=4, index=0, jmax=3, hmax=2)
    c, temp = 0.5, 1.2
    hist = sa.metropolis_histogram(J, h, c, temp, 3_000_000, seed=9)
    states = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1) * 2 - 1
    e = pimi.energy(J, h, states.T.astype(np.int64)).astype(np.float64)
    p = np.exp(-c * (e - e.min()) / temp)
    p /= p.sum()
    q = hist / hist.sum()
    assert 0.5 * np.abs(p - q).sum() < 0.01
    # and not the law of the neighbouring mistakes
    for wrong in (np.exp(+c * (e - e.min()) / temp), np.exp(-(e - e.min()) / temp)):
        wrong = wrong / wrong.sum()
        assert 0.5 * np.abs(wrong - q).sum() > 0.05


def test_sk200_scale_sanity():
    """SK energies per N^(3/2) approach the Parisi value -0.763 (sanity only)."""
    J, h = w.sk1(200, seed=1, index=0)
    e, s, _ = sa.anneal(J, h, 1 / math.sqrt(200), runs=1)
    assert -0.80 < e / 200 ** 1.5 < -0.70
    assert pimi.energy(J, h, s.astype(np.int64)) == e


def test_rejects_invalid():
    J, h = w.sk1(8, seed=1, index=0)
    bad = J.copy()
    bad[0, 1] = 3
    with pytest.raises(ValueError):
        sa.anneal(bad, h, 0.5)
    with pytest.raises(ValueError):
        sa.anneal(J, h, 0.0)
