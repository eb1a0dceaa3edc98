"""Pins of Eq. (1)/(2) and the brute-force ground state."""
import itertools

import numpy as np
import pytest

import workloads as w
from oracle import pimi, ground


def _loop_energy(J, h, s):
    n = len(s)
    e = 0
    for i in range(n):
        for j in range(i + 1, n):
            e -= int(J[i][j]) * int(s[i]) * int(s[j])
        e -= int(h[i]) * int(s[i])
    return e


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_energy_matches_python_double_loop(n):
    J, h = w.random_int8(n, seed=3, index=n, jmax=9, hmax=7)
    rng = np.random.default_rng(n)
    for _ in range(20):
        s = rng.choice([-1, 1], size=n)
        assert pimi.energy(J, h, s) == _loop_energy(J, h, s)


def test_field_form_equals_eq1_batch():
    J, h = w.random_int8(37, seed=5, jmax=127, hmax=1000)
    s = np.random.default_rng(0).choice([-1, 1], size=(37, 50))
    I = pimi.local_field(J, h, s)
    np.testing.assert_array_equal(pimi.energy_from_field(I, h, s), pimi.energy(J, h, s))
    np.testing.assert_array_equal(pimi.energy(J, h, s),
                                  [pimi.energy(J, h, s[:, k]) for k in range(50)])


def test_local_field_is_eq2():
    J, h = w.random_int8(6, seed=2, jmax=5, hmax=3)
    s = np.array([1, -1, -1, 1, 1, -1])
    for i in range(6):
        assert pimi.local_field(J, h, s)[i] == sum(int(J[i][j]) * s[j] for j in range(6)) + h[i]


def test_maxcut_energy_is_edges_minus_twice_cut():
    J, h = w.maxcut(30, seed=9)
    A = -J.astype(np.int64)
    m = int(np.triu(A, 1).sum())
    rng = np.random.default_rng(1)
    for _ in range(20):
        s = rng.choice([-1, 1], size=30)
        cut = sum(int(A[i, j]) for i in range(30) for j in range(i + 1, 30) if s[i] != s[j])
        assert pimi.energy(J, h, s) == m - 2 * cut


def test_f64_energy_equals_int_energy_on_integers():
    J, h = w.random_int8(12, seed=4, jmax=20, hmax=5)
    s = np.random.default_rng(3).choice([-1, 1], size=(12, 7))
    np.testing.assert_array_equal(pimi.energy_f64(J, h, s), pimi.energy(J, h, s).astype(float))


@pytest.mark.parametrize("n", [3, 6, 10])
def test_brute_force_matches_itertools(n):
    J, h = w.random_int8(n, seed=8, index=n, jmax=4, hmax=3)
    energies = [pimi.energy(J, h, np.array(c)) for c in itertools.product([-1, 1], repeat=n)]
    e, s, count = ground.brute_force(J, h)
    assert e == min(energies)
    assert count == energies.count(min(energies))
    assert pimi.energy(J, h, s) == e


@pytest.mark.parametrize("n", [4, 7, 12])
def test_brute_force_closed_forms(n):
    # ferromagnet on the complete graph: all-aligned, E = -N(N-1)/2, two minimisers
    J = np.ones((n, n), dtype=np.int8) - np.eye(n, dtype=np.int8)
    e, _, count = ground.brute_force(J, np.zeros(n, np.int32))
    assert e == -n * (n - 1) // 2 and count == 2
    # complete antiferromagnet: H = ((sum s)^2 - N) / 2, minimised at |sum s| <= 1
    e, _, count = ground.brute_force(-J, np.zeros(n, np.int32))
    from math import comb
    if n % 2 == 0:
        assert e == -n // 2 and count == comb(n, n // 2)
    else:
        assert e == (1 - n) // 2 and count == 2 * comb(n, n // 2)
    # free spins in a field: E = -sum |h_i|
    h = np.arange(1, n + 1, dtype=np.int32) * np.where(np.arange(n) % 2, 1, -1)
    e, s, count = ground.brute_force(np.zeros((n, n), np.int8), h)
    assert e == -int(np.abs(h).sum()) and count == 1
    np.testing.assert_array_equal(s, np.sign(h))


def test_sk20_ground_state_fixture():
    """SK-1 N=20 (seed 1, instance 0): ground-state energy by enumeration of
    all 2^20 states.  The stored value was written by
    tests/golden/make_golden.py, which calls only the oracle."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sk20_ground.json")))
    J, h = w.sk1(20, seed=gold["seed"], index=gold["index"])
    e, s, count = ground.brute_force(J, h)
    assert e == gold["e_gs"] and count == gold["count"]
