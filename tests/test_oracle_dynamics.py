"""Statistical and structural pins of the oracle's update loops.

* Sequential heat bath (Eq. (3) with exact tanh, U(-1,1) noise, eta = 1):
  P(s_i = +1) = (1 + tanh(beta I_i)) / 2, whose stationary law is the Boltzmann
  distribution exp(-beta H) (textbook Gibbs sampler).
* Synchronous heat bath (Box 1 middle, same choices): Little dynamics, whose
  stationary law is pi(s) ~ exp(beta h.s) prod_i cosh(beta I_i(s)) (Peretto).
* Spec dynamics (LUT, inertia, table noise) on N = 3: the empirical one-step
  transitions driven by Philox match the exact transition matrix obtained by
  enumerating every noise index.
* Special cases: frozen dynamics under large inertia; J = 0 single-spin chains
  against the Gaussian CDF; resume equivalence; the sequential rule touches only
  spin t mod N.
"""
import itertools

import numpy as np
import pytest
from scipy.stats import norm

import workloads as w
from oracle import pimi


def _states(n):
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.int64)


def _hist(S):
    n = S.shape[0]
    idx = ((S > 0).astype(np.int64) * (1 << np.arange(n)[::-1, None])).sum(0)
    return np.bincount(idx, minlength=1 << n) / S.shape[1]


def _tv(p, q):
    return 0.5 * np.abs(p - q).sum()


def _exact_problem(J, h):
    # c = 1 so that the tanh argument is beta * I; xi = 0; table unused
    return pimi.Problem(J, h, c=1.0, xi=0.0, levels=4, ztab=np.zeros(256))


def _uniform_noise(seed):
    rng = np.random.default_rng(seed)
    return lambda shape, step: rng.uniform(-1.0, 1.0, size=shape)


J4 = np.array([[0, 1, -2, 1], [1, 0, 1, -1], [-2, 1, 0, 2], [1, -1, 2, 0]], dtype=np.int8)
H4 = np.array([1, -1, 0, 2], dtype=np.int32)


def test_sequential_heat_bath_is_boltzmann():
    beta = 0.35
    prob = _exact_problem(J4, H4)
    R, sweeps = 30000, 60
    T = sweeps * 4
    res = pimi.run_sequential(prob, np.full(T, beta), np.ones(T), seed=0, stream=0,
                              trials=np.arange(R), act=np.tanh, noise=_uniform_noise(1))
    S = _states(4)
    e = np.array([pimi.energy(J4, H4, s) for s in S], dtype=np.float64)
    p = np.exp(-beta * e)
    p /= p.sum()
    assert _tv(_hist(res["final"]), p) < 0.02
    # a wrong sign of beta (or of the field) would give a very different law
    q = np.exp(beta * e)
    q /= q.sum()
    assert _tv(p, q) > 0.2


def test_parallel_heat_bath_is_little_dynamics():
    beta = 0.3
    prob = _exact_problem(J4, H4)
    R, T = 30000, 60
    res = pimi.run_parallel(prob, np.full(T, beta), np.ones(T), seed=0, stream=0,
                            trials=np.arange(R), act=np.tanh, noise=_uniform_noise(2))
    S = _states(4)
    I = pimi.local_field(J4, H4, S.T)
    logpi = beta * (H4 @ S.T) + np.log(np.cosh(beta * I)).sum(0)
    pi = np.exp(logpi - logpi.max())
    pi /= pi.sum()
    assert _tv(_hist(res["final"]), pi) < 0.02
    # ...and it is not the Boltzmann law of the same model
    e = np.array([pimi.energy(J4, H4, s) for s in S], dtype=np.float64)
    b = np.exp(-beta * e)
    b /= b.sum()
    assert _tv(pi, b) > 0.05


def _spec_transition_matrix(prob, beta, eta):
    """Exact P(s' | s) for the spec dynamics by enumerating every noise index."""
    n = prob.n
    S = _states(n)
    P = np.zeros((len(S), len(S)))
    u = np.arange(1 << prob.bits)
    for a, s in enumerate(S):
        I = pimi.local_field(prob.J, prob.h, s)
        act = pimi.tanh_lut((beta * prob.c) * I, prob.levels)
        p_up = np.array([
            (pimi.spin_decision(act[i], np.full(u.size, s[i]), prob.xi, eta, prob.ztab[u]) == 1).mean()
            for i in range(n)])
        for b, s2 in enumerate(S):
            P[a, b] = np.prod(np.where(s2 > 0, p_up, 1 - p_up))
    return P


def test_spec_dynamics_transitions_match_exact_matrix():
    J = np.array([[0, 2, -1], [2, 0, 1], [-1, 1, 0]], dtype=np.int8)
    h = np.array([1, 0, -1], dtype=np.int32)
    prob = pimi.Problem(J, h, c=0.4, xi=0.3, levels=4, ztab=w.gauss_table(8))
    beta, eta = 1.0, 0.8
    P = _spec_transition_matrix(prob, beta, eta)
    np.testing.assert_allclose(P.sum(1), 1.0)
    R, T = 4096, 40
    s = pimi.initial_spins(5, 0, np.arange(R), 3)
    counts = np.zeros_like(P)
    S = _states(3)
    code = lambda X: ((X > 0).astype(np.int64) * np.array([[4], [2], [1]])).sum(0)
    for t in range(T):
        res = pimi.run_parallel(prob, [beta], [eta], seed=5, stream=0, trials=np.arange(R),
                                init=s, start_step=t)
        s2 = res["final"]
        np.add.at(counts, (code(s), code(s2)), 1)
        s = s2
    # chi-square per source state with enough visits
    for a in range(8):
        n_a = counts[a].sum()
        if n_a < 500:
            continue
        exp = P[a] * n_a
        mask = exp > 5
        chi2 = ((counts[a][mask] - exp[mask]) ** 2 / exp[mask]).sum()
        dof = max(1, mask.sum() - 1)
        assert chi2 < dof + 6 * np.sqrt(2 * dof) + 10, (a, chi2, dof)


def test_large_inertia_freezes_the_state():
    J, h = w.sk1(12, seed=4)
    ztab = w.gauss_table(8)
    eta = 0.1  # eta * max|Z| = 0.29 < xi - 1
    prob = pimi.Problem(J, h, c=1.0, xi=1.5, levels=4, ztab=ztab)
    res = pimi.run_parallel(prob, np.full(50, 2.0), np.full(50, eta), seed=3, stream=0,
                            trials=np.arange(16), trace=True)
    s0 = pimi.initial_spins(3, 0, np.arange(16), 12)
    np.testing.assert_array_equal(res["final"], s0)
    assert np.all(res["trace"] == res["trace"][0])
    assert np.all(res["t_best"] == 0)


@pytest.mark.parametrize("xi,eta", [(0.0, 0.5), (0.2, 1.0), (0.5, 0.7)])
def test_free_spins_flip_with_gaussian_probability(xi, eta):
    """J = 0, h = 0: the table input is 0, which the half-open bins map to the
    level +1/3 (L = 4).  P(s' = +1 | s) = P(1/3 + xi s + eta Z > 0), i.e. the
    normal CDF at (1/3 + xi s) / eta up to the 8-bit quantisation of Z."""
    n = 64
    prob = pimi.Problem(np.zeros((n, n), np.int8), np.zeros(n, np.int32), c=1.0, xi=xi,
                        levels=4, ztab=w.gauss_table(8))
    R = 256
    s = pimi.initial_spins(9, 0, np.arange(R), n)
    up = {1: [0, 0], -1: [0, 0]}
    for t in range(30):
        s2 = pimi.run_parallel(prob, [1.0], [eta], seed=9, stream=0, trials=np.arange(R),
                               init=s, start_step=t)["final"]
        for sv in (1, -1):
            m = s == sv
            up[sv][0] += int((s2[m] == 1).sum())
            up[sv][1] += int(m.sum())
        s = s2
    for sv in (1, -1):
        p_hat = up[sv][0] / up[sv][1]
        p = norm.cdf((1 / 3 + xi * sv) / eta)
        sd = np.sqrt(p * (1 - p) / up[sv][1])
        assert abs(p_hat - p) < 4 * sd + 1.5 / 256, (sv, p_hat, p)


def test_resume_equals_uninterrupted_run():
    J, h = w.maxcut(24, seed=2)
    prob = pimi.Problem(J, h, c=2 / np.sqrt(24), xi=0.7, levels=4, ztab=w.gauss_table(8))
    beta = w.linear_beta(200)
    eta = w.eta_sqrt_beta_over_5(beta)
    trials = np.arange(8)
    full = pimi.run_parallel(prob, beta, eta, 11, 3, trials, target=-60)
    a = pimi.run_parallel(prob, beta[:120], eta[:120], 11, 3, trials, target=-60)
    b = pimi.run_parallel(prob, beta[120:], eta[120:], 11, 3, trials, init=a["final"],
                          start_step=120, target=-60)
    np.testing.assert_array_equal(b["final"], full["final"])
    best = np.minimum(a["e_best"], b["e_best"])
    np.testing.assert_array_equal(best, full["e_best"])
    fh = np.where(a["first_hit"] >= 0, a["first_hit"], b["first_hit"])
    np.testing.assert_array_equal(fh, full["first_hit"])


def test_sequential_updates_only_spin_t_mod_n():
    J, h = w.sk1(7, seed=1)
    prob = pimi.Problem(J, h, c=1.0, xi=0.0, levels=4, ztab=w.uniform_table(8))
    s = pimi.initial_spins(2, 0, np.arange(32), 7)
    for t in range(20):
        s2 = pimi.run_sequential(prob, [0.5], [1.0], 2, 0, np.arange(32), init=s,
                                 start_step=t)["final"]
        changed = np.any(s2 != s, axis=1)
        assert not np.any(np.delete(changed, t % 7))
        s = s2


def test_pimi_reaches_sk20_ground_states():
    """All 16 SK-1 N=20 instances of the parity workload: PIMI with the spec
    dynamics reaches the brute-force ground energy on most trials."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sk20_ground_all.json")))
    beta = w.linear_beta(1000)
    eta = w.eta_sqrt_beta_over_5(beta)
    for g in gold[:4]:
        J, h = w.sk1(20, seed=g["seed"], index=g["index"])
        prob = pimi.Problem(J, h, c=1 / np.sqrt(20), xi=0.5, levels=4, ztab=w.gauss_table(8))
        res = pimi.run_parallel(prob, beta, eta, 1, g["index"], np.arange(64), target=g["e_gs"])
        assert res["e_best"].min() == g["e_gs"]
        assert np.all(res["e_best"] >= g["e_gs"])
        assert (res["first_hit"] >= 0).mean() > 0.5


def test_exact_tie_keeps_the_current_spin():
    """Reading for sign(0): a decision argument that is exactly zero keeps
    s_i(t).  With J = 0 the table gives +1/3, and xi = 1/3 with no noise makes
    the argument exactly 0 for s = -1 and 2/3 for s = +1: a frozen state."""
    n = 16
    prob = pimi.Problem(np.zeros((n, n), np.int8), np.zeros(n, np.int32), c=1.0, xi=1.0 / 3.0,
                        levels=4, ztab=w.gauss_table(8))
    res = pimi.run_parallel(prob, np.ones(5), np.zeros(5), seed=4, stream=0, trials=np.arange(8))
    np.testing.assert_array_equal(res["final"], pimi.initial_spins(4, 0, np.arange(8), n))
    # without inertia every spin goes to +1 (argument 1/3 > 0)
    prob0 = pimi.Problem(np.zeros((n, n), np.int8), np.zeros(n, np.int32), c=1.0, xi=0.0,
                         levels=4, ztab=w.gauss_table(8))
    res0 = pimi.run_parallel(prob0, np.ones(1), np.zeros(1), seed=4, stream=0, trials=np.arange(8))
    assert np.all(res0["final"] == 1)
