"""Pins for the MIMO detection reference (oracle/mimo.py) and the real-valued
mode of the PIMI oracle.

Each test checks the oracle against something the mathematics fixes, not
against itself: the complex product, the residual identity of the
perturbation mapping evaluated with the independent Eq. (1) energy, exhaustive
ML search, the MMSE solution computed by a second route, exact recovery at
vanishing noise, and the exact scale invariance of the update rule.
"""
import numpy as np
import pytest

import workloads as w
from oracle import mimo, pimi

RNG = np.random.default_rng(20260417)


def _complex(shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def test_gray_labelling_roundtrip_and_adjacency():
    for qam in (4, 16, 64):
        k = w.mimo.bits_per_symbol(qam) // 2
        allb = np.array([[(g >> (k - 1 - i)) & 1 for i in range(k)] for g in range(1 << k)])
        lv = w.mimo.levels_from_bits(allb, qam)
        assert sorted(lv.tolist()) == w.mimo.pam_levels(qam).tolist()
        assert np.array_equal(w.mimo.bits_from_levels(lv, qam), allb)
        order = np.argsort(lv)
        for a, b in zip(order[:-1], order[1:]):  # neighbouring levels differ in one bit
            assert np.count_nonzero(allb[a] != allb[b]) == 1


def test_real_equivalent_is_the_complex_product():
    H, x = _complex((5, 3)), _complex(3)
    Hr, yr = mimo.real_equivalent(H, H @ x)
    assert np.allclose(Hr @ mimo.real_vector(x), yr, rtol=0, atol=1e-12)
    assert np.isclose(np.linalg.norm(yr), np.linalg.norm(H @ x), rtol=1e-14)
    assert np.allclose(mimo.complex_vector(mimo.real_vector(x)), x, rtol=0, atol=0)


@pytest.mark.parametrize("mode,qam", [("ml", 4), ("ml", 16), ("di", 4), ("di", 16)])
def test_residual_identity(mode, qam):
    """||y - H(xm + T s)||^2 = E_Eq1(s) + const for every s, with E from the
    double-sum form of Eq. (1) (pin P11)."""
    p = w.mimo.mimo_problem(6, 6, qam, 12.0, seed=3, index=1)
    d = mimo.detector_instance(p, mode)
    n = d["J"].shape[0]
    assert n == (2 * 6 if (mode, qam) == ("ml", 4) else 4 * 6)
    assert np.array_equal(d["J"], d["J"].T) and np.all(np.diag(d["J"]) == 0)
    for _ in range(20):
        s = RNG.choice([-1.0, 1.0], size=n)
        resid = d["y"] - d["H"] @ (d["xm"] + d["T"] @ s)
        lhs = float(resid @ resid)
        rhs = pimi.energy_f64(d["J"], d["h"], s) + d["const"]
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-9)
    # the field I = J s + h is minus the gradient of the residual in s
    s = RNG.choice([-1.0, 1.0], size=n)
    HT = d["H"] @ d["T"]
    grad = 2.0 * HT.T @ (HT @ s - (d["y"] - d["H"] @ d["xm"]))
    G = HT.T @ HT
    I = pimi.local_field_f64(d["J"], d["h"], s)
    assert np.allclose(I, -(grad - 2.0 * np.diag(G) * s), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("qam,nt", [(4, 4), (16, 2)])
def test_ising_ground_state_is_ml(qam, nt):
    """Brute force over spins (the Ising side) and over symbol vectors (the ML
    definition) select the same vector."""
    for idx in range(3):
        p = w.mimo.mimo_problem(nt, nt, qam, 8.0, seed=5, index=idx)
        d = mimo.detector_instance(p, "ml")
        n = d["J"].shape[0]
        states = np.array(list(np.ndindex(*(2,) * n)), dtype=np.float64).T * 2 - 1  # [n, 2^n]
        e = pimi.energy_f64(d["J"], d["h"], states)
        s_best = states[:, int(np.argmin(e))]
        x_ising = mimo.decode(d["xm"], d["T"], s_best, qam)
        x_ml, dist = mimo.ml_enumerate(p["H"], p["y"], qam)
        assert np.array_equal(x_ising, x_ml)
        assert float(np.min(e)) + d["const"] == pytest.approx(dist, rel=1e-10)


def test_ml_recovers_transmitted_at_high_snr():
    for idx in range(3):
        p = w.mimo.mimo_problem(3, 3, 16, 60.0, seed=9, index=idx)
        x_ml, _ = mimo.ml_enumerate(p["H"], p["y"], 16)
        assert np.array_equal(x_ml, p["x"])


def test_mmse_two_routes_and_noise_free_recovery():
    p = w.mimo.mimo_problem(8, 8, 16, 15.0, seed=2, index=4)
    z = mimo.mmse(p["H"], p["y"], p["esn0"])
    # real-valued route: (H^T H + I / (Es/N0)) zr = H^T y in the real model
    Hr, yr = mimo.real_equivalent(p["H"], p["y"])
    zr = np.linalg.solve(Hr.T @ Hr + np.eye(Hr.shape[1]) / p["esn0"], Hr.T @ yr)
    assert np.allclose(mimo.real_vector(z), zr, rtol=1e-10, atol=1e-10)
    # without noise and with a vanishing regulariser MMSE inverts the channel
    H = p["H"]
    x = p["x"]
    assert np.allclose(mimo.mmse(H, H @ x, 1e14), x, atol=1e-6)
    assert np.array_equal(mimo.mmse_detect(H, H @ x, 1e14, 16), x)


def test_slicing():
    v = np.array([-9.0, -3.2, -2.0, -0.1, 0.0, 0.9, 1.99, 2.0, 3.5, 8.0])
    assert mimo.slice_levels(v, 16).tolist() == [-3, -3, -1, -1, 1, 1, 1, 3, 3, 3]
    assert mimo.slice_levels(v, 4).tolist() == [-1, -1, -1, -1, 1, 1, 1, 1, 1, 1]


@pytest.mark.parametrize("mode,qam", [("ml", 4), ("ml", 16), ("di", 16)])
def test_decode_of_transmitted_spins(mode, qam):
    """A spin vector that encodes the transmitted symbols decodes to them."""
    p = w.mimo.mimo_problem(5, 5, qam, 30.0, seed=4, index=2)
    d = mimo.detector_instance(p, mode)
    n2 = 10
    target = mimo.real_vector(p["x"]) - d["xm"]
    wts = mimo.transform_weights(mode, qam)
    if mode == "ml" and qam == 4:
        s = target
    elif mode == "ml":  # x = 2 s1 + s2 with s1, s2 = +-1
        s1 = np.where(target > 0, 1.0, -1.0)
        s = np.concatenate([s1, target - 2.0 * s1])
    else:  # d = s1 + s2 in {-2, 0, 2}; only when the MMSE guess is one step away
        if np.any(np.abs(target) > 2):
            pytest.skip("MMSE estimate more than one level away")
        s1 = np.where(target >= 0, 1.0, -1.0)
        s = np.concatenate([s1, target - s1])
    assert len(wts) * n2 == len(s) and set(np.unique(s)) <= {-1.0, 1.0}
    assert np.array_equal(mimo.decode(d["xm"], d["T"], s, qam), p["x"])


def test_real_mode_is_exactly_scale_invariant():
    """A real instance J/8, h/8 with coupling scale 8c makes the same binary64
    decisions as the integer instance (J, h, c): g' = 8 fl(beta c) and
    g' I' = g I exactly, so trajectories agree bit for bit and energies scale
    by 1/8."""
    J, h = w.random_int8(24, seed=6, index=0, jmax=5, hmax=7)
    c = 1.0 / np.sqrt(24)
    ztab = w.gauss_table(8)
    beta = w.linear_beta(60, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    pi = pimi.Problem(J, h, c, 0.5, 4, ztab)
    pr = pimi.RealProblem(J.astype(np.float64) / 8.0, h.astype(np.float64) / 8.0, 8.0 * c, 0.5, 4, ztab)
    a = pimi.run_parallel(pi, beta, eta, 11, 3, np.arange(16), trace=True)
    b = pimi.run_parallel(pr, beta, eta, 11, 3, np.arange(16), trace=True)
    assert np.array_equal(a["final"], b["final"])
    assert np.array_equal(a["t_best"], b["t_best"])
    assert np.array_equal(a["best_state"], b["best_state"])
    assert np.array_equal(a["trace"].astype(np.float64) / 8.0, b["trace"])
    sa = pimi.run_sequential(pi, beta, eta, 11, 3, np.arange(4))
    sb = pimi.run_sequential(pr, beta, eta, 11, 3, np.arange(4))
    assert np.array_equal(sa["final"], sb["final"])
    assert np.array_equal(sa["e_best"].astype(np.float64) / 8.0, sb["e_best"])


def test_real_field_energy_matches_eq1():
    p = w.mimo.mimo_problem(4, 4, 16, 10.0, seed=1, index=0)
    d = mimo.detector_instance(p, "di")
    s = RNG.choice([-1.0, 1.0], size=(d["J"].shape[0], 7))
    I = pimi.local_field_f64(d["J"], d["h"], s)
    assert np.allclose(pimi.energy_from_field_f64(I, d["h"], s), pimi.energy_f64(d["J"], d["h"], s),
                       rtol=1e-12, atol=1e-9)
