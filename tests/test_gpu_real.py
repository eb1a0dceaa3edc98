"""GPU parity of the real-valued path (FP8 / BF16 MFMA and plain FP32 kernels).

Exact cases: couplings and fields that are dyadic with few significant bits
(J = 2^-k * q with q exact in the operand format, h a multiple of the same
power of two) make every binary32 operation of the kernels exact, so the
trajectories must equal the binary64 oracle's bit for bit: final spins, best
energy, its step, the state there, first hit.

MIMO cases (arbitrary reals): the binary64 energy of every returned state
equals the oracle's binary64 energy of that state within 1e-9 relative, and
the detection quality (symbol error rate) of the quantised kernels is
statistically indistinguishable from the binary64 oracle's dynamics.
"""
import numpy as np
import pytest

import workloads as w
from oracle import mimo, pimi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _dyadic(n, prec, seed, with_h):
    """Symmetric J with zero diagonal whose quantisation is exact, and h."""
    rng = np.random.default_rng([seed, n])
    if prec == "fp8":
        q = rng.integers(-16, 17, size=(n, n)).astype(np.float64)  # exact in e4m3
        q = np.triu(q, 1)
        q = q + q.T
        if n >= 2:
            q[0, 1] = q[1, 0] = 448.0  # max |q| = 448 -> scale 2^-6 exactly
        J = q * 2.0 ** -6
    else:
        q = rng.integers(-200, 201, size=(n, n)).astype(np.float64)  # 8 significant bits
        q = np.triu(q, 1)
        q = q + q.T
        J = q * 2.0 ** -5
    h = rng.integers(-1000, 1001, size=n) * 2.0 ** -6 if with_h else np.zeros(n)
    return J, h


def _schedule(kind, steps):
    if kind == "mimo":
        return w.constant(steps, 1.0), w.mimo_eta(steps, 0.05, 1.0), 1.0, 2.0
    beta = w.linear_beta(steps, 0.1, 3.0)
    return beta, w.eta_sqrt_beta_over_5(beta), 0.37, 0.5


CASES = [
    # prec, kernel, n, trials, steps, with_h, schedule
    ("fp8", "mfma", 16, 32, 40, True, "mimo"),
    ("fp8", "mfma", 33, 40, 60, False, "anneal"),
    ("fp8", "mfma", 64, 128, 50, True, "mimo"),
    ("fp8", "mfma", 100, 70, 60, True, "anneal"),
    ("fp8", "mfma", 256, 64, 30, True, "mimo"),
    ("bf16", "mfma", 16, 32, 40, True, "mimo"),
    ("bf16", "mfma", 63, 40, 60, False, "anneal"),
    ("bf16", "mfma", 128, 96, 40, True, "mimo"),
    ("bf16", "mfma", 200, 33, 40, True, "anneal"),
    ("bf16", "mfma", 256, 32, 30, False, "mimo"),
    ("fp8", "plain", 33, 40, 60, True, "anneal"),
    ("bf16", "plain", 128, 64, 40, True, "mimo"),
    ("fp8", "mfma", 64, 1, 30, True, "mimo"),      # a single trial
    ("bf16", "mfma", 96, 40, 1, True, "mimo"),     # a single step
    ("bf16", "plain", 40, 1, 30, False, "anneal"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_dyadic_trajectories_bit_exact(gpu_lib, case):
    prec, kernel, n, trials, steps, with_h, sched = case
    _say(f"real dyadic prec={prec} kernel={kernel} n={n} trials={trials} steps={steps} h={with_h} {sched}")
    pim = gpu_lib
    ztab = w.gauss_table(8)
    beta, eta, c, xi = _schedule(sched, steps)
    count = 2
    insts, refs = [], []
    for k in range(count):
        J, h = _dyadic(n, prec, seed=11 + k, with_h=with_h)
        Jq, scale = pim.quantize(J, prec)
        assert np.array_equal(Jq, J) and scale == 2.0 ** np.round(np.log2(scale))
        insts.append(pim.Instance(J, h, j_scale=c, xi=xi, levels=4, noise_table=ztab, rng_stream=5 + k,
                                  prec=prec))
        refs.append((J, h))
    batch = pim.Batch(insts, trials)
    targets = [float(pimi.energy_f64(J, h, np.ones(n))) - 1.0 for (J, h) in refs]
    batch.run(beta, eta, seed=21, kernel=kernel, target=targets)
    for k, (J, h) in enumerate(refs):
        prob = pimi.RealProblem(J, h, c, xi, 4, ztab)
        ref = pimi.run_parallel(prob, beta, eta, 21, 5 + k, np.arange(trials), target=targets[k])
        got = batch.trials_of(k)
        np.testing.assert_array_equal(got["final"], ref["final"].T.astype(np.int8))
        np.testing.assert_array_equal(got["t_best"], ref["t_best"])
        np.testing.assert_array_equal(got["e_best"], ref["e_best"])
        np.testing.assert_array_equal(got["best_state"], ref["best_state"].T.astype(np.int8))
        np.testing.assert_array_equal(got["first_hit"], ref["first_hit"])
        spins, e, trial, step = batch.best(k)
        e_ref = pimi.energy_f64(J, h, ref["best_state"].astype(np.float64))
        assert e == pytest.approx(float(e_ref.min()), rel=1e-12)
        assert int(np.argmin(e_ref)) == trial or e_ref[trial] == e_ref.min()
    batch.close()


# (prec, n, instances, trials, steps, with_h): instances x ceil(trials / 32)
# trial blocks > 128, so the launch takes the batched form (one wave per
# 32-trial block, every row tile of the block in that wave)
BATCHED = [
    ("fp8", 64, 5, 1024, 40, True),      # 2 row tiles: one K step of the FP8 MFMA
    ("fp8", 200, 5, 1000, 30, True),     # 7 tiles, ragged N and a ragged last block
    ("fp8", 96, 9, 500, 30, False),      # 3 tiles (odd), 16 blocks per instance
    ("bf16", 128, 5, 1024, 30, True),    # 4 tiles
    ("bf16", 256, 5, 1024, 24, False),   # 8 tiles, the largest N
    ("bf16", 33, 5, 1000, 40, True),     # 2 tiles, 1 spin in the second
]


@pytest.mark.parametrize("case", BATCHED, ids=lambda c: "-".join(map(str, c)))
def test_dyadic_batched_form_bit_exact(gpu_lib, case):
    """The batched one-wave-per-block form, the one that large batches and
    large server chunks run, against the binary64 oracle bit for bit."""
    prec, n, count, trials, steps, with_h = case
    assert count * ((trials + 31) // 32) > 128
    _say(f"real dyadic batched form prec={prec} n={n} instances={count} trials={trials} steps={steps}")
    pim = gpu_lib
    ztab = w.gauss_table(8)
    beta, eta, c, xi = _schedule("anneal", steps)
    insts, refs = [], []
    for k in range(count):
        J, h = _dyadic(n, prec, seed=40 + k, with_h=with_h)
        insts.append(pim.Instance(J, h, j_scale=c, xi=xi, levels=4, noise_table=ztab, rng_stream=60 + k,
                                  prec=prec))
        refs.append((J, h))
    batch = pim.Batch(insts, trials)
    targets = [float(pimi.energy_f64(J, h, np.ones(n))) - 1.0 for (J, h) in refs]
    batch.run(beta, eta, seed=31, target=targets)
    for k, (J, h) in enumerate(refs):
        prob = pimi.RealProblem(J, h, c, xi, 4, ztab)
        ref = pimi.run_parallel(prob, beta, eta, 31, 60 + k, np.arange(trials), target=targets[k])
        got = batch.trials_of(k)
        np.testing.assert_array_equal(got["final"], ref["final"].T.astype(np.int8))
        np.testing.assert_array_equal(got["t_best"], ref["t_best"])
        np.testing.assert_array_equal(got["e_best"], ref["e_best"])
        np.testing.assert_array_equal(got["best_state"], ref["best_state"].T.astype(np.int8))
        np.testing.assert_array_equal(got["first_hit"], ref["first_hit"])
        spins, e, trial, step = batch.best(k)
        e_ref = pimi.energy_f64(J, h, ref["best_state"].astype(np.float64))
        assert e == float(e_ref.min()) and trial == int(np.argmin(e_ref))
        np.testing.assert_array_equal(spins, ref["best_state"][:, trial].astype(np.int8))
    batch.close()


@pytest.mark.parametrize("prec", ["fp8", "bf16"])
def test_real_resume_equals_uninterrupted(gpu_lib, prec):
    _say(f"real resume prec={prec}")
    pim = gpu_lib
    n, trials, steps = 48, 64, 40
    J, h = _dyadic(n, prec, seed=3, with_h=True)
    ztab = w.gauss_table(8)
    beta, eta, c, xi = _schedule("mimo", steps)
    inst = pim.Instance(J, h, j_scale=c, xi=xi, noise_table=ztab, rng_stream=9, prec=prec)
    full = pim.Batch([inst], trials).run(beta, eta, seed=4)
    part = pim.Batch([inst], trials).run(beta[:15], eta[:15], seed=4)
    mid = part.trials_of(0)["final"]
    rest = pim.Batch([inst], trials, init_spins=mid[None]).run(beta[15:], eta[15:], seed=4, start_step=15)
    np.testing.assert_array_equal(rest.trials_of(0)["final"], full.trials_of(0)["final"])


def _mimo_instances(pim, nt, qam, db, count, prec, seed=1):
    probs, insts, maps = [], [], []
    for k in range(count):
        p = w.mimo.mimo_problem(nt, nt, qam, db, seed=seed, index=k)
        J, h, xm = pim.mimo_ising(p["H"], p["y"], qam, "di", p["esn0"])
        probs.append(p)
        maps.append((J, h, xm))
        insts.append(pim.Instance(J, h, j_scale=1.0, xi=2.0, noise_table=w.gauss_table(8), rng_stream=k,
                                  prec=prec))
    return probs, insts, maps


@pytest.mark.parametrize("prec", ["fp8", "bf16"])
def test_mimo_energies_are_binary64(gpu_lib, prec):
    """Pin P14: the energy pim_best reports for the returned state equals the
    oracle's binary64 Eq. (1) energy of that state; pim_energy likewise."""
    _say(f"mimo energies prec={prec}")
    pim = gpu_lib
    probs, insts, maps = _mimo_instances(pim, 8, 16, 15.0, 12, prec)
    steps = 32
    beta, eta = w.constant(steps, 1.0), w.mimo_eta(steps, 0.05, 1.0)
    batch = pim.Batch(insts, 32).run(beta, eta, seed=5)
    rng = np.random.default_rng(3)
    for k, (J, h, xm) in enumerate(maps):
        spins, e, trial, step = batch.best(k)
        e_ref = pimi.energy_f64(J, h, spins.astype(np.float64))
        assert e == pytest.approx(e_ref, rel=1e-9, abs=1e-9)
        trials = batch.trials_of(k)
        e_all = pimi.energy_f64(J, h, trials["best_state"].T.astype(np.float64))
        assert e == pytest.approx(e_all.min(), rel=1e-9, abs=1e-9)  # argmin over trials
        S = rng.choice(np.array([-1, 1], np.int8), size=(5, J.shape[0]))
        np.testing.assert_allclose(insts[k].energy(S), pimi.energy_f64(J, h, S.T.astype(np.float64)),
                                   rtol=1e-12, atol=1e-9)
    batch.close()


@pytest.mark.parametrize("prec,kernel", [("fp8", "mfma"), ("bf16", "mfma"), ("fp8", "plain")])
def test_mimo_detection_matches_oracle_statistically(gpu_lib, prec, kernel):
    """8x8 16-QAM at 15 dB, DI mapping, 32 trials x 32 steps, 256 channels
    (2048 symbols): the symbol error rate of the GPU kernels is within three
    standard deviations of the binary64 oracle's dynamics on the same channels
    (different arithmetic, so in effect different noise realisations of the
    same law).  The deviation is that of the difference of two independent
    binomial rates at the pooled rate, which overstates the spread of these
    correlated runs; there is no additive allowance."""
    _say(f"mimo SER prec={prec} kernel={kernel}")
    pim = gpu_lib
    count, nt, qam = 256, 8, 16
    probs, insts, maps = _mimo_instances(pim, nt, qam, 15.0, count, prec, seed=2)
    steps = 32
    beta, eta = w.constant(steps, 1.0), w.mimo_eta(steps, 0.05, 1.0)
    batch = pim.Batch(insts, 32).run(beta, eta, seed=6, kernel=kernel)
    err_gpu = err_orc = 0
    for k, p in enumerate(probs):
        J, h, xm = maps[k]
        spins, e, _, _ = batch.best(k)
        err_gpu += mimo.symbol_errors(p["x"], pim.mimo_decode(xm, spins, qam, "di"))
        d = mimo.detector_instance(p, "di")
        prob = pimi.RealProblem(d["J"], d["h"], 1.0, 2.0, 4, w.gauss_table(8))
        ref = pimi.run_parallel(prob, beta, eta, 6, k, np.arange(32))
        e_ref = pimi.energy_f64(d["J"], d["h"], ref["best_state"].astype(np.float64))
        s_ref = ref["best_state"][:, int(np.argmin(e_ref))]
        err_orc += mimo.symbol_errors(p["x"], mimo.decode(d["xm"], d["T"], s_ref, qam))
    total = count * nt
    assert total >= 2000
    ser_gpu, ser_orc = err_gpu / total, err_orc / total
    pooled = (err_gpu + err_orc) / (2 * total)
    sd = np.sqrt(2 * pooled * (1 - pooled) / total)
    print(f"SER gpu {ser_gpu:.4f} oracle {ser_orc:.4f} over {total} symbols, 3 sd = {3 * sd:.4f}", flush=True)
    assert abs(ser_gpu - ser_orc) <= 3 * sd
    batch.close()


@pytest.mark.parametrize("prec,nt", [("fp8", 16), ("bf16", 16), ("fp8", 32), ("fp8", 48), ("bf16", 48)])
def test_latency_and_batched_forms_agree(gpu_lib, prec, nt):
    """A launch with few 32-trial blocks runs the latency form (the block's row
    tiles split over several waves, spins exchanged through LDS); a launch
    with many runs one wave per block.  The same MIMO instances (arbitrary
    reals) run both ways give identical trajectories, best states, steps and
    binary32 energies."""
    _say(f"latency vs batched forms prec={prec} Nt={nt}")
    pim = gpu_lib
    count, trials, steps = 40, 128, 48  # 160 blocks together: the batched form
    probs, insts, maps = _mimo_instances(pim, nt, 16, 18.0, count, prec, seed=8)
    beta, eta = w.constant(steps, 1.0), w.mimo_eta(steps, 0.05, 1.0)
    big = pim.Batch(insts, trials).run(beta, eta, seed=9)
    for k0 in range(0, count, 8):  # 8 instances x 4 blocks = 32 blocks: the latency form
        small = pim.Batch(insts[k0:k0 + 8], trials).run(beta, eta, seed=9)
        for j in range(8):
            a, b = big.trials_of(k0 + j), small.trials_of(j)
            for key in ("final", "best_state", "e_best", "t_best", "e_final"):
                np.testing.assert_array_equal(a[key], b[key], err_msg=f"{key} instance {k0 + j}")
        small.close()
    big.close()
