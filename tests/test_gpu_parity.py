"""GPU parity: the HIP kernels against the CPU oracle, element by element.

Integer instances must reproduce the oracle bit for bit: final spins, best
energy, its step, the state there, first hit, final energy.  Every case prints
its name before touching the GPU.
"""
import numpy as np
import pytest

import workloads as w
from oracle import pimi

pytestmark = pytest.mark.gpu

KERNELS = ["mfma", "plain"]


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _oracle(J, h, c, xi, L, ztab, beta, eta, seed, stream, trials, init=None, start=0, target=None):
    prob = pimi.Problem(J, h, c=c, xi=xi, levels=L, ztab=ztab)
    return pimi.run_parallel(prob, beta, eta, seed, stream, np.asarray(trials), init=init,
                             start_step=start, target=target)


def _compare(batch, k, ref, trials, n):
    got = batch.trials_of(k)
    idx = np.asarray(trials)
    np.testing.assert_array_equal(got["final"][idx], ref["final"].T.astype(np.int8))
    np.testing.assert_array_equal(got["e_best"][idx], ref["e_best"].astype(np.float64))
    np.testing.assert_array_equal(got["t_best"][idx], ref["t_best"])
    np.testing.assert_array_equal(got["best_state"][idx], ref["best_state"].T.astype(np.int8))
    np.testing.assert_array_equal(got["first_hit"][idx], ref["first_hit"])
    return got


def _run_case(pim, kind, n, trials, steps, kernel, seed=7, count=1, xi=0.5, noise="gauss",
              hmax=0, jmax=1, init=False, c=None, stream_base=3, beta1=3.0):
    insts, probs = [], []
    ztab = w.gauss_table(8) if noise == "gauss" else w.uniform_table(8)
    for k in range(count):
        if kind == "sk":
            J, h = w.sk1(n, seed=seed, index=k)
        elif kind == "maxcut":
            J, h = w.maxcut(n, seed=seed, index=k)
        else:
            J, h = w.random_int8(n, seed=seed, index=k, jmax=jmax, hmax=hmax)
        cc = c if c is not None else 1.0 / np.sqrt(n)
        insts.append(pim.Instance(J, h, j_scale=cc, xi=xi, levels=4, noise_table=ztab,
                                  rng_stream=stream_base + k))
        probs.append((J, h, cc))
    init_spins = None
    if init:
        init_spins = np.random.default_rng(seed).choice([-1, 1], size=(count, trials, n)).astype(np.int8)
    beta = w.linear_beta(steps, 0.1, beta1)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, trials, init_spins=init_spins)
    targets = []
    for (J, h, cc) in probs:
        targets.append(int(pimi.energy(J, h, np.ones(n, dtype=np.int64))) - 1)
    batch.run(beta, eta, seed=seed, kernel=kernel, target=targets)
    for k, (J, h, cc) in enumerate(probs):
        ref = _oracle(J, h, cc, xi, 4, ztab, beta, eta, seed, stream_base + k, np.arange(trials),
                      init=None if init_spins is None else init_spins[k].T.astype(np.int64),
                      target=targets[k])
        _compare(batch, k, ref, np.arange(trials), n)
    return batch


@pytest.mark.parametrize("kernel", KERNELS)
def test_sk20_config_parity(gpu_lib, kernel):
    """SK-1 N=20, 64 trials x 1000 steps, beta linear 0.1 -> 3.0 (first
    workload), four instances of the sixteen."""
    _say(f"sk20 64x1000 kernel={kernel}")
    _run_case(gpu_lib, "sk", 20, 64, 1000, kernel, seed=1, count=4)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n,trials", [(1, 8), (31, 40), (32, 64), (33, 33), (200, 70), (256, 32), (50, 1), (2, 1)])
def test_sizes_and_ragged_tails(gpu_lib, kernel, n, trials):
    _say(f"sizes n={n} trials={trials} kernel={kernel}")
    _run_case(gpu_lib, "maxcut" if n > 2 else "sk", n, trials, 120, kernel, seed=n, count=2)


@pytest.mark.parametrize("kernel", ["mfma", "f4"])
def test_instances_not_a_multiple_of_the_xcd_count(gpu_lib, kernel):
    """Eleven instances of three trial blocks each, the last block ragged: the
    LDS kernels place an instance's blocks on one XCD (workgroup b runs
    instance b mod 8 + 8 floor((b / 8) / blocks), the grid padded to whole
    groups of 8 instances), so every (instance, block) pair must run exactly
    once.  Every trial of every instance against the oracle."""
    _say(f"11 instances x 300 trials kernel={kernel}")
    _run_case(gpu_lib, "sk", 40, 300, 60, kernel, seed=13, count=11)


@pytest.mark.parametrize("kernel", KERNELS)
def test_general_int8_with_fields(gpu_lib, kernel):
    _say(f"int8 couplings with h kernel={kernel}")
    _run_case(gpu_lib, "int8", 45, 48, 200, kernel, seed=5, count=2, jmax=100, hmax=900, c=0.004, xi=0.3)


@pytest.mark.parametrize("kernel", KERNELS)
def test_conventional_parallel_uniform_noise(gpu_lib, kernel):
    _say(f"conventional parallel (xi=0, uniform) kernel={kernel}")
    _run_case(gpu_lib, "sk", 60, 32, 150, kernel, seed=9, xi=0.0, noise="uniform")


@pytest.mark.parametrize("kernel", KERNELS)
def test_caller_initial_spins(gpu_lib, kernel):
    _say(f"caller initial spins kernel={kernel}")
    _run_case(gpu_lib, "maxcut", 70, 36, 100, kernel, seed=11, count=2, init=True, xi=0.7)


def test_resume_equals_uninterrupted(gpu_lib):
    _say("resume 2 x 150 == 300")
    pim = gpu_lib
    n, R = 90, 64
    J, h = w.sk1(n, seed=4)
    ztab = w.gauss_table(8)
    mk = lambda: pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=2)
    beta = w.linear_beta(300)
    eta = w.eta_sqrt_beta_over_5(beta)
    i0 = mk()
    full = pim.Batch([i0], R).run(beta, eta, seed=3).trials_of(0)
    a = pim.Batch([i0], R).run(beta[:150], eta[:150], seed=3).trials_of(0)
    b = pim.Batch([i0], R, init_spins=a["final"][None]).run(beta[150:], eta[150:], seed=3,
                                                             start_step=150).trials_of(0)
    np.testing.assert_array_equal(b["final"], full["final"])
    np.testing.assert_array_equal(np.minimum(a["e_best"], b["e_best"]), full["e_best"])


def test_energy_f64_matches_eq1(gpu_lib):
    _say("pim_energy binary64")
    pim = gpu_lib
    for n in (5, 64, 200, 256):
        J, h = w.random_int8(n, seed=n, jmax=60 if n < 100 else 1, hmax=50)
        inst = pim.Instance(J, h, j_scale=0.01, xi=0.5)
        S = np.random.default_rng(n).choice([-1, 1], size=(37, n)).astype(np.int8)
        got = inst.energy(S)
        want = pimi.energy(J, h, S.T.astype(np.int64)).astype(np.float64)
        np.testing.assert_array_equal(got, want)
        # the same configurations from device memory, read in place
        import torch
        dev = torch.from_numpy(S).to("cuda")
        np.testing.assert_array_equal(inst.energy(dev), want)
        np.testing.assert_array_equal(inst.energy(dev[5:9]), want[5:9])


def test_best_is_lowest_trial_argmin(gpu_lib):
    _say("pim_best argmin")
    pim = gpu_lib
    n, R = 24, 96
    J, h = w.sk1(n, seed=12)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=w.gauss_table(8))
    batch = pim.Batch([inst], R)
    beta = w.linear_beta(400)
    batch.run(beta, w.eta_sqrt_beta_over_5(beta), seed=5)
    tr = batch.trials_of(0)
    spins, e, trial, step = batch.best(0)
    assert e == tr["e_best"].min()
    assert trial == int(np.flatnonzero(tr["e_best"] == e)[0])
    assert step == tr["t_best"][trial]
    np.testing.assert_array_equal(spins, tr["best_state"][trial])
    assert pimi.energy(J, h, spins.astype(np.int64)) == e


def test_cancel_reports_partial_results(gpu_lib):
    _say("cancel")
    pim = gpu_lib
    n, R = 64, 64
    J, h = w.sk1(n, seed=2)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5)
    batch = pim.Batch([inst], R)
    T = 200000
    beta = np.full(T, 1.0)
    batch.run(beta, np.full(T, 0.4), seed=1)
    batch.cancel()
    with pytest.raises(pim.PimError) as ei:
        batch.trials_of(0)
    assert ei.value.status == pim.PIM_ERR_CANCELLED
    # a new run on the same batch clears the request and completes
    batch.run(beta[:50], np.full(50, 0.4), seed=1)
    batch.trials_of(0)


def test_full_size_maxcut200_sampled_trials(gpu_lib):
    """Max-Cut N=200, 1024 trials x 10^4 steps (second workload) in the launch
    configuration the benchmark uses; the oracle recomputes three sampled
    trials in full, and every trial's best state must have the energy the
    kernel tracked."""
    _say("maxcut200 1024x10000 mfma, sampled oracle trials")
    pim = gpu_lib
    n, R, T = 200, 1024, 10000
    J, h = w.maxcut(n, seed=1, index=0)
    ztab = w.gauss_table(8)
    c = 2.0 / np.sqrt(n)
    inst = pim.Instance(J, h, j_scale=c, xi=0.7, noise_table=ztab, rng_stream=0)
    beta = w.linear_beta(T)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch([inst], R)
    batch.run(beta, eta, seed=1, kernel="mfma")
    got = batch.trials_of(0)
    sample = np.array([0, 517, 1023])
    ref = _oracle(J, h, c, 0.7, 4, ztab, beta, eta, 1, 0, sample)
    np.testing.assert_array_equal(got["final"][sample], ref["final"].T.astype(np.int8))
    np.testing.assert_array_equal(got["e_best"][sample], ref["e_best"])
    np.testing.assert_array_equal(got["t_best"][sample], ref["t_best"])
    e_states = pimi.energy(J, h, got["best_state"].T.astype(np.int64))
    np.testing.assert_array_equal(e_states, got["e_best"])
    e_final = pimi.energy(J, h, got["final"].T.astype(np.int64))
    np.testing.assert_array_equal(e_final, got["e_final"])


def test_full_size_sk200_batched_sampled(gpu_lib):
    """Batched SK-1 N=200, 128 instances x 1024 trials x 10^4 steps with a
    first-hit target: the benchmark's headline workload in its launch
    configuration.  The oracle recomputes sampled (instance, trial) pairs in
    full; every trial's tracked best and final energies equal the energies of
    the states returned, and each instance's best is the lowest trial."""
    _say("sk200 128x1024x10000 mfma, sampled oracle trials")
    pim = gpu_lib
    n, R, T, I = 200, 1024, 10000, 128
    c, xi, ztab = 1.0 / np.sqrt(n), 0.5, w.gauss_table(8)
    target = -2000.0
    probs = [w.sk1(n, seed=1, index=k) for k in range(I)]
    insts = [pim.Instance(J, h, j_scale=c, xi=xi, levels=4, noise_table=ztab, rng_stream=k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, R)
    batch.run(beta, eta, seed=1, kernel="mfma", target=[target] * I)
    for k, trials in ((0, [0, 1023]), (63, [5, 700]), (127, [511])):
        J, h = probs[k]
        ref = _oracle(J, h, c, xi, 4, ztab, beta, eta, 1, k, trials, target=target)
        _compare(batch, k, ref, trials, n)
    for k in range(I):
        J, h = probs[k]
        got = batch.trials_of(k)
        for key, ek in (("best_state", "e_best"), ("final", "e_final")):
            S = got[key].T.astype(np.int64)
            np.testing.assert_array_equal(pimi.energy_from_field(pimi.local_field(J, h, S), h, S), got[ek])
        hit = got["first_hit"]
        assert np.all((hit == -1) == (got["e_best"] > target))
        spins, e, trial, _ = batch.best(k)
        assert e == got["e_best"].min() and trial == int(np.argmin(got["e_best"]))
    batch.close()


def test_full_size_uneven_batch_sampled(gpu_lib):
    """The benchmark's uneven-N workload as it is launched there: 128 SK-1
    instances with N_k = [100, 200, 400, 800, 1000][k mod 5], 1024 trials x
    2000 steps, tuned, one graph launch, with first-hit targets.  The oracle
    recomputes a sampled trial of six instances (every N) in full; every
    trial's tracked best energy equals the energy of its returned state."""
    _say("uneven N 128x1024x2000 graph, sampled oracle trials")
    pim = gpu_lib
    sizes = [100, 200, 400, 800, 1000]
    count, R, T = 128, 1024, 2000
    ns = [sizes[k % 5] for k in range(count)]
    ztab = w.gauss_table(8)
    probs = [w.sk1(ns[k], seed=9, index=k) for k in range(count)]
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(ns[k]), xi=0.5, noise_table=ztab, rng_stream=k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    tgt = [float(np.floor(-0.7 * n ** 1.5)) for n in ns]
    batch = pim.Batch(insts, R)
    batch.tune(steps=100)
    batch.run(beta, eta, seed=2, target=tgt)
    for k, trials in ((0, [0]), (1, [1023]), (2, [300]), (3, [511]), (4, [1000]), (124, [7])):
        J, h = probs[k]
        ref = _oracle(J, h, 1 / np.sqrt(ns[k]), 0.5, 4, ztab, beta, eta, 2, k, trials, target=tgt[k])
        _compare(batch, k, ref, trials, ns[k])
    for k in range(count):
        J, h = probs[k]
        got = batch.trials_of(k)
        S = got["best_state"].T.astype(np.int64)
        np.testing.assert_array_equal(pimi.energy_from_field(pimi.local_field(J, h, S), h, S), got["e_best"])
        assert np.all((got["first_hit"] == -1) == (got["e_best"] > tgt[k]))
    batch.close()


SEQ_CASES = [
    # n, trials, steps, hmax, jmax, xi, noise
    (20, 64, 2000, 0, 1, 0.0, "uniform"),
    (1, 8, 12, 0, 1, 0.0, "uniform"),
    (33, 40, 1, 2, 2, 0.5, "gauss"),     # a single step
    (33, 70, 700, 5, 3, 0.5, "gauss"),
    (64, 64, 640, 0, 1, 0.0, "uniform"),
    (200, 16, 600, 0, 1, 0.0, "uniform"),
    (256, 40, 520, 2, 1, 0.7, "gauss"),
]


@pytest.mark.parametrize("case", SEQ_CASES, ids=lambda c: "-".join(map(str, c)))
def test_sequential_kernel_parity(gpu_lib, case):
    """Conventional PIM with sequential updates (one spin per step) against
    the oracle's sequential dynamics, bit for bit."""
    n, trials, steps, hmax, jmax, xi, noise = case
    _say(f"sequential n={n} trials={trials} steps={steps} h={hmax} xi={xi} {noise}")
    pim = gpu_lib
    ztab = w.gauss_table(8) if noise == "gauss" else w.uniform_table(8)
    J, h = w.random_int8(n, seed=12, index=n, jmax=jmax, hmax=hmax)
    c = 1.0 / np.sqrt(n)
    beta = w.constant(steps, 0.8)
    eta = w.conventional_eta(steps, 1.5, 0.05)
    inst = pim.Instance(J, h, j_scale=c, xi=xi, noise_table=ztab, rng_stream=2)
    batch = pim.Batch([inst], trials)
    target = int(pimi.energy(J, h, np.ones(n, dtype=np.int64))) - 1
    batch.run(beta, eta, seed=9, kernel="seq", target=[target], start_step=3)
    prob = pimi.Problem(J, h, c=c, xi=xi, levels=4, ztab=ztab)
    ref = pimi.run_sequential(prob, beta, eta, 9, 2, np.arange(trials), start_step=3, target=target)
    _compare(batch, 0, ref, np.arange(trials), n)
    batch.close()


def test_sequential_resume(gpu_lib):
    _say("sequential resume")
    pim = gpu_lib
    n, trials = 40, 64
    J, h = w.sk1(n, seed=2, index=1)
    ztab = w.uniform_table(8)
    beta, eta = w.constant(300, 0.5), w.conventional_eta(300, 1.0, 0.1)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.0, noise_table=ztab, rng_stream=4)
    full = pim.Batch([inst], trials).run(beta, eta, seed=3, kernel="seq")
    part = pim.Batch([inst], trials).run(beta[:111], eta[:111], seed=3, kernel="seq")
    rest = pim.Batch([inst], trials, init_spins=part.trials_of(0)["final"][None]).run(
        beta[111:], eta[111:], seed=3, kernel="seq", start_step=111)
    np.testing.assert_array_equal(rest.trials_of(0)["final"], full.trials_of(0)["final"])


@pytest.mark.parametrize("xi", [0.0, 0.5])
def test_recorded_states_and_flip_rate(gpu_lib, xi):
    """Every recorded state s(t) equals the oracle's, and the device's
    neighbour-triggered flip counts equal the oracle's definition exactly."""
    from oracle import diagnostics
    _say(f"record states + P_NT xi={xi}")
    pim = gpu_lib
    n, trials, steps = 40, 70, 90
    J, h = w.maxcut(n, seed=4, index=2)
    ztab = w.gauss_table(8)
    c = 2 / np.sqrt(n)
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    inst = pim.Instance(J, h, j_scale=c, xi=xi, noise_table=ztab, rng_stream=6)
    batch = pim.Batch([inst], trials).run(beta, eta, seed=2, record=True)
    prob = pimi.Problem(J, h, c=c, xi=xi, levels=4, ztab=ztab)
    ref = pimi.run_parallel(prob, beta, eta, 2, 6, np.arange(trials), record=True)
    for a in (0, 31, 32, trials - 1):
        np.testing.assert_array_equal(batch.states(0, a), ref["states"][:, :, a])
    num, den = batch.flip_counts(0)
    rnum, rden = diagnostics.neighbor_flip_counts(J, ref["states"])
    np.testing.assert_array_equal(num, rnum)
    np.testing.assert_array_equal(den, rden)
    batch.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_single_step_runs(gpu_lib, kernel):
    """T = 1: one update and the energies of s(0) and s(1), bit-exact."""
    _say(f"single step {kernel}")
    _run_case(gpu_lib, "int", 40, 33, 1, kernel, seed=21, count=2, jmax=2, hmax=2)


def test_schedule_changes_between_runs(gpu_lib):
    """Runs of one batch with changing schedules: the same one twice, one that
    differs only in its last beta, one that differs only in its first eta, a
    shorter one, then the first again.  Every run is bit-exact against the
    oracle, on a single-N batch and on an uneven-N (graph) batch, so step tables
    kept on the device are reused only for an identical schedule."""
    pim = gpu_lib
    ztab = w.gauss_table(8)
    beta_a = w.linear_beta(120, 0.1, 3.0)
    eta_a = w.eta_sqrt_beta_over_5(beta_a)
    beta_b = beta_a.copy()
    beta_b[-1] += 0.25
    eta_d = eta_a.copy()
    eta_d[0] *= 0.5
    scheds = [("A", beta_a, eta_a), ("A again", beta_a, eta_a), ("last beta changed", beta_b, eta_a),
              ("A", beta_a, eta_a), ("first eta changed", beta_a, eta_d),
              ("shorter", beta_a[:60].copy(), eta_a[:60].copy()), ("A", beta_a, eta_a)]
    for ns in ([40, 40], [20, 64]):
        trials = 48
        probs, insts = [], []
        for k, n in enumerate(ns):
            J, h = w.random_int8(n, seed=61, index=k, jmax=2, hmax=2)
            c = 1.0 / np.sqrt(n)
            probs.append((J, h, c))
            insts.append(pim.Instance(J, h, j_scale=c, xi=0.5, noise_table=ztab, rng_stream=70 + k))
        batch = pim.Batch(insts, trials)
        targets = [float(pimi.energy(J, h, np.ones(len(h), dtype=np.int64))) - 1 for (J, h, c) in probs]
        for name, beta, eta in scheds:
            _say(f"schedule change, N {ns}: {name}")
            batch.run(beta, eta, seed=5, target=targets)
            for k, (J, h, c) in enumerate(probs):
                ref = _oracle(J, h, c, 0.5, 4, ztab, beta, eta, 5, 70 + k, np.arange(trials), target=targets[k])
                _compare(batch, k, ref, np.arange(trials), len(h))
        batch.close()


def test_kernel_changes_between_runs(gpu_lib):
    """One batch, one schedule, alternating kernels: int8 MFMA, plain FP32,
    sequential (which reads the same cached step tables as the MFMA kernel),
    then int8 MFMA again.  The parallel runs match the oracle's parallel
    dynamics and the sequential run its sequential dynamics, bit for bit."""
    pim = gpu_lib
    n, trials = 40, 48
    ztab = w.gauss_table(8)
    J, h = w.random_int8(n, seed=62, index=0, jmax=2, hmax=2)
    c = 1.0 / np.sqrt(n)
    beta = w.linear_beta(100, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    inst = pim.Instance(J, h, j_scale=c, xi=0.5, noise_table=ztab, rng_stream=9)
    batch = pim.Batch([inst], trials)
    target = int(pimi.energy(J, h, np.ones(n, dtype=np.int64))) - 1
    par = _oracle(J, h, c, 0.5, 4, ztab, beta, eta, 6, 9, np.arange(trials), target=target)
    prob = pimi.Problem(J, h, c=c, xi=0.5, levels=4, ztab=ztab)
    seq = pimi.run_sequential(prob, beta, eta, 6, 9, np.arange(trials), target=target)
    for kernel, ref in (("mfma", par), ("plain", par), ("seq", seq), ("mfma", par), ("seq", seq)):
        _say(f"kernel change: {kernel}")
        batch.run(beta, eta, seed=6, kernel=kernel, target=[target])
        _compare(batch, 0, ref, np.arange(trials), n)
    batch.close()


def test_run_on_another_stream(gpu_lib):
    """A long run of a batch on one stream, then at once a run with another
    schedule on a second stream: the second waits for the first and equals
    the same run done alone, bit for bit."""
    import ctypes
    import torch
    _say("runs of one batch on two streams")
    pim = gpu_lib
    n = 64
    J, h = w.random_int8(n, seed=72, index=0, jmax=2, hmax=2)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=w.gauss_table(8), rng_stream=90)
    b1 = w.linear_beta(20000, 0.1, 3.0)
    b2 = w.linear_beta(3000, 0.2, 2.5)
    e1, e2 = w.eta_sqrt_beta_over_5(b1), w.eta_sqrt_beta_over_5(b2)
    alone = pim.Batch([inst], 256).run(b2, e2, seed=14)
    ref = alone.trials_of(0)
    alone.close()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    batch = pim.Batch([inst], 256)
    batch.run(b1, e1, seed=14, stream=ctypes.c_void_p(s1.cuda_stream))
    batch.run(b2, e2, seed=14, stream=ctypes.c_void_p(s2.cuda_stream))
    got = batch.trials_of(0)
    for key in ("final", "e_best", "t_best", "best_state", "first_hit"):
        assert np.array_equal(got[key], ref[key]), key
    batch.close()


def test_concurrent_runs_on_distinct_batches(gpu_lib):
    """Two threads run two batches at once, each on its own stream, switching
    schedules every run so that every run compiles and uploads its step tables
    through the library's shared staging buffer.  Every run equals the result
    of the same run done alone, bit for bit."""
    import threading
    import torch
    _say("concurrent runs on distinct batches")
    pim = gpu_lib
    ztab = w.gauss_table(8)
    jobs = []
    for k, (n, T) in enumerate(((40, 90), (72, 60))):
        J, h = w.random_int8(n, seed=71, index=k, jmax=2, hmax=2)
        inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=80 + k)
        b1 = w.linear_beta(T, 0.1, 3.0)
        b2 = w.linear_beta(T, 0.2, 2.5)
        scheds = [(b1, w.eta_sqrt_beta_over_5(b1)), (b2, w.eta_sqrt_beta_over_5(b2))]
        refs = []
        for beta, eta in scheds:
            alone = pim.Batch([inst], 48).run(beta, eta, seed=13)
            refs.append(alone.trials_of(0))
            alone.close()
        jobs.append((inst, scheds, refs))
    errors = []

    def worker(inst, scheds, refs):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                batch = pim.Batch([inst], 48)
                for it in range(8):
                    beta, eta = scheds[it % 2]
                    batch.run(beta, eta, seed=13)
                    got = batch.trials_of(0)
                    for key in ("final", "e_best", "t_best", "best_state"):
                        if not np.array_equal(got[key], refs[it % 2][key]):
                            errors.append((inst.n, it, key))
                batch.close()
        except Exception as e:  # noqa: BLE001 - reported by the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=job) for job in jobs]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors


def test_uneven_n_batch_one_graph(gpu_lib):
    """Instances of different N in one batch (one graph launch per run): every
    instance bit-exact against the oracle, with caller initial spins for some
    and a repeated run giving identical results."""
    _say("uneven N batch (graph)")
    pim = gpu_lib
    ns = [20, 200, 33, 64, 100, 20]
    trials, steps = 70, 150
    ztab = w.gauss_table(8)
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    probs, insts = [], []
    for k, n in enumerate(ns):
        J, h = w.random_int8(n, seed=31, index=k, jmax=2, hmax=3 if k % 2 else 0)
        c = 1.0 / np.sqrt(n)
        probs.append((J, h, c))
        insts.append(pim.Instance(J, h, j_scale=c, xi=0.5, noise_table=ztab, rng_stream=40 + k))
    rng = np.random.default_rng(8)
    init = [rng.choice([-1, 1], size=(trials, n)).astype(np.int8) for n in ns]
    batch = pim.Batch(insts, trials, init_spins=init)
    targets = [float(pimi.energy(J, h, np.ones(len(h), dtype=np.int64))) - 1 for (J, h, c) in probs]
    for rep in range(2):
        batch.run(beta, eta, seed=17, target=targets)
        for k, (J, h, c) in enumerate(probs):
            ref = _oracle(J, h, c, 0.5, 4, ztab, beta, eta, 17, 40 + k, np.arange(trials),
                          init=init[k].T.astype(np.int64), target=targets[k])
            _compare(batch, k, ref, np.arange(trials), len(h))
    assert batch.kernel_ms() > 0
    spins, e, trial, step = batch.best(1)
    assert len(spins) == 200 and e == pimi.energy(probs[1][0], probs[1][1], spins.astype(np.int64))
    batch.close()


def test_tune_keeps_trajectories(gpu_lib):
    _say("autotune waves per workgroup")
    pim = gpu_lib
    ns = [64, 200]
    trials, steps = 300, 120
    ztab = w.gauss_table(8)
    insts, probs = [], []
    for k, n in enumerate(ns):
        J, h = w.sk1(n, seed=3, index=k)
        insts.append(pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=k))
        probs.append((J, h, 1 / np.sqrt(n)))
    batch = pim.Batch(insts, trials)
    waves = batch.tune(steps=50)
    assert len(waves) == 2 and set(waves.tolist()) <= {1, 2, 4}
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch.run(beta, eta, seed=5)
    for k, (J, h, c) in enumerate(probs):
        ref = _oracle(J, h, c, 0.5, 4, ztab, beta, eta, 5, k, np.arange(trials))
        _compare(batch, k, ref, np.arange(trials), len(h))
    batch.close()


BIG_CASES = [
    # n, trials, steps, jmax, hmax
    (257, 64, 60, 3, 0),
    (300, 40, 50, 1, 5),
    (512, 33, 40, 2, 0),
    (600, 130, 30, 2, 3),   # three row tiles per wave; a second, mostly idle trial block
    (700, 200, 20, 1, 0),
    (777, 64, 30, 1, 0),
    (1000, 32, 30, 1, 0),
    (1024, 70, 24, 30, 40),
    (300, 1, 20, 2, 1),     # a single trial: one column block with 31 empty lanes, 3 empty blocks
    (400, 64, 1, 2, 0),     # a single step
]


@pytest.mark.parametrize("case", BIG_CASES, ids=lambda c: "-".join(map(str, c)))
def test_streamed_large_n_parity(gpu_lib, case):
    """N > 256: couplings streamed from global memory by eight waves that
    share 128 trials' spins in LDS (two, three or four row tiles per wave,
    partial trial blocks, fields); bit-exact against the oracle."""
    n, trials, steps, jmax, hmax = case
    _say(f"large N streamed n={n} trials={trials} steps={steps}")
    batch = _run_case(gpu_lib, "int", n, trials, steps, "mfma", seed=13, count=2, jmax=jmax, hmax=hmax)
    # the re-rank: pim_best returns the trial whose best state has the lowest
    # Eq. (1) energy (ties to the lowest trial), with that energy and state
    for k in range(2):
        J, h = w.random_int8(n, seed=13, index=k, jmax=jmax, hmax=hmax)
        got = batch.trials_of(k)
        e_all = pimi.energy(J, h, got["best_state"].T.astype(np.int64))
        spins, e, trial, step = batch.best(k)
        assert e == float(e_all.min())
        assert trial == int(np.argmin(e_all))
        np.testing.assert_array_equal(spins, got["best_state"][trial])
        assert step == got["t_best"][trial]


def test_mixed_small_and_large_n_graph(gpu_lib):
    _say("mixed small/large N in one graph")
    pim = gpu_lib
    ns = [100, 400, 200, 1000]
    trials, steps = 48, 40
    ztab = w.gauss_table(8)
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    probs, insts = [], []
    for k, n in enumerate(ns):
        J, h = w.sk1(n, seed=21, index=k)
        probs.append((J, h, 1 / np.sqrt(n)))
        insts.append(pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=k))
    batch = pim.Batch(insts, trials).run(beta, eta, seed=2)
    for k, (J, h, c) in enumerate(probs):
        ref = _oracle(J, h, c, 0.5, 4, ztab, beta, eta, 2, k, np.arange(trials))
        _compare(batch, k, ref, np.arange(trials), len(h))
        spins, e, trial, step = batch.best(k)
        assert e == pimi.energy(J, h, spins.astype(np.int64))
    batch.close()
