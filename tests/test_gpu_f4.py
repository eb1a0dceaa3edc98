"""GPU parity of the streamed sweep on e2m1 (FP4) operands (N > 256, couplings
in {0, +-1, +-2, +-3, +-4, +-6}) against the CPU oracle, bit for bit: the
field is the same exact integer as in the int8 kernel, so final spins, best
energy, its step and state, and the first hit must all equal the oracle's.
Every case prints its name before touching the GPU."""
import numpy as np
import pytest

import workloads as w
from oracle import pimi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _oracle(J, h, c, beta, eta, seed, stream, trials, ztab, init=None, start=0, target=None):
    prob = pimi.Problem(J, h, c=c, xi=0.5, levels=4, ztab=ztab)
    return pimi.run_parallel(prob, beta, eta, seed, stream, np.asarray(trials), init=init, start_step=start,
                             target=target)


def _compare(got, ref, trials):
    idx = np.asarray(trials)
    np.testing.assert_array_equal(got["final"][idx], ref["final"].T.astype(np.int8))
    np.testing.assert_array_equal(got["e_best"][idx], ref["e_best"].astype(np.float64))
    np.testing.assert_array_equal(got["t_best"][idx], ref["t_best"])
    np.testing.assert_array_equal(got["best_state"][idx], ref["best_state"].T.astype(np.int8))
    np.testing.assert_array_equal(got["first_hit"][idx], ref["first_hit"])


def _e2m1_instance(n, seed, index, values, hmax=0):
    """Symmetric J with entries drawn from `values`, zero diagonal."""
    rng = np.random.default_rng([seed, index, 77])
    J = np.zeros((n, n), np.int8)
    iu = np.triu_indices(n, 1)
    J[iu] = rng.choice(np.asarray(values, np.int8), size=iu[0].size)
    J = (J + J.T).astype(np.int8)
    h = rng.integers(-hmax, hmax + 1, size=n).astype(np.int32) if hmax else np.zeros(n, np.int32)
    return J, h


def _run(pim, probs, trials, steps, kernel, seed, init=None, start=0, beta1=3.0):
    ztab = w.gauss_table(8)
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, levels=4, noise_table=ztab, rng_stream=3 + k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(steps, 0.1, beta1)
    eta = w.eta_sqrt_beta_over_5(beta)
    targets = [int(pimi.energy(J, h, np.ones(len(h), dtype=np.int64))) - 1 for J, h in probs]
    batch = pim.Batch(insts, trials, init_spins=init)
    batch.run(beta, eta, seed=seed, kernel=kernel, target=targets, start_step=start)
    return batch, beta, eta, targets, ztab


CASES = [
    # n, trials, steps, values, hmax
    (257, 64, 60, (-1, 0, 1), 0),                  # nine row tiles: odd K-step count, padded half step
    (300, 40, 50, (-1, 1), 5),                     # fields
    (400, 64, 1, (-2, -1, 0, 1, 2), 0),            # a single step
    (512, 33, 40, (-3, -1, 1, 3), 0),
    (600, 130, 30, (-4, -2, 0, 2, 4), 3),          # three row tiles per wave; a mostly idle trial block
    (777, 64, 30, (-6, -4, -3, -2, -1, 0, 1, 2, 3, 4, 6), 0),  # every e2m1 integer
    (1000, 32, 30, (-1, 1), 0),
    (1024, 70, 24, (-6, 6, -1, 1), 40),
    (300, 1, 20, (-1, 0, 1), 1),                   # a single trial
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}-{len(c[3])}v-h{c[4]}")
def test_f4_streamed_parity(gpu_lib, case):
    n, trials, steps, values, hmax = case
    _say(f"f4 streamed n={n} trials={trials} steps={steps} values={values} hmax={hmax}")
    probs = [_e2m1_instance(n, 31, k, values, hmax) for k in range(2)]
    batch, beta, eta, targets, ztab = _run(gpu_lib, probs, trials, steps, "f4", seed=13)
    for k, (J, h) in enumerate(probs):
        got = batch.trials_of(k)
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 13, 3 + k, np.arange(trials), ztab, target=targets[k])
        _compare(got, ref, np.arange(trials))
        e_all = pimi.energy(J, h, got["best_state"].T.astype(np.int64))
        spins, e, trial, step = batch.best(k)
        assert e == float(e_all.min()) and trial == int(np.argmin(e_all))
    batch.close()


def test_f4_equals_int8_and_initial_spins(gpu_lib):
    """The same batch through both kernels, from caller spins: identical
    results, and both equal to the oracle on sampled trials."""
    _say("f4 vs int8, caller initial spins, n=800")
    pim = gpu_lib
    n, trials, steps = 800, 96, 40
    probs = [w.sk1(n, seed=5, index=k) for k in range(3)]
    init = np.random.default_rng(4).choice([-1, 1], size=(3, trials, n)).astype(np.int8)
    b4, beta, eta, targets, ztab = _run(pim, probs, trials, steps, "f4", seed=9, init=init)
    b8, *_ = _run(pim, probs, trials, steps, "mfma", seed=9, init=init)
    for k, (J, h) in enumerate(probs):
        g4, g8 = b4.trials_of(k), b8.trials_of(k)
        for key in ("final", "e_best", "t_best", "best_state", "first_hit", "e_final"):
            np.testing.assert_array_equal(g4[key], g8[key], err_msg=key)
        tr = [0, 95] if k != 1 else [41]
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 9, 3 + k, tr, ztab, init=init[k][tr].T.astype(np.int64),
                      target=targets[k])
        _compare(g4, ref, tr)
    b4.close()
    b8.close()


def test_f4_resume_equals_uninterrupted(gpu_lib):
    _say("f4 resume 2 x 40 == 80, n=448")
    pim = gpu_lib
    n, R = 448, 64
    J, h = w.sk1(n, seed=6)
    ztab = w.gauss_table(8)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=2)
    beta = w.linear_beta(80)
    eta = w.eta_sqrt_beta_over_5(beta)
    full = pim.Batch([inst], R).run(beta, eta, seed=3, kernel="f4").trials_of(0)
    a = pim.Batch([inst], R).run(beta[:40], eta[:40], seed=3, kernel="f4").trials_of(0)
    b = pim.Batch([inst], R, init_spins=a["final"][None]).run(beta[40:], eta[40:], seed=3, start_step=40,
                                                              kernel="f4").trials_of(0)
    np.testing.assert_array_equal(b["final"], full["final"])
    np.testing.assert_array_equal(np.minimum(a["e_best"], b["e_best"]), full["e_best"])


def test_f4_ineligible_couplings_fall_back(gpu_lib):
    """A coupling of 5 has no exact e2m1 code: the batch runs the int8 kernel
    and still equals the oracle."""
    _say("f4 request with |J| = 5: int8 kernel, n=300")
    n, trials, steps = 300, 32, 30
    probs = [_e2m1_instance(n, 8, k, (-5, -1, 1, 5)) for k in range(2)]
    batch, beta, eta, targets, ztab = _run(gpu_lib, probs, trials, steps, "f4", seed=4)
    for k, (J, h) in enumerate(probs):
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 4, 3 + k, np.arange(trials), ztab, target=targets[k])
        _compare(batch.trials_of(k), ref, np.arange(trials))
    batch.close()


def test_f4_mixed_sizes_graph(gpu_lib):
    """Uneven N in one graph launch with the e2m1 kernel: parts with N <= 256
    run the int8 LDS kernel, the others the e2m1 streamed kernel."""
    _say("f4 mixed small/large N graph")
    pim = gpu_lib
    ns = [100, 400, 200, 1000, 800]
    trials, steps = 48, 40
    probs = [w.sk1(n, seed=21, index=k) for k, n in enumerate(ns)]
    ztab = w.gauss_table(8)
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, noise_table=ztab, rng_stream=k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, trials).run(beta, eta, seed=2, kernel="f4")
    for k, (J, h) in enumerate(probs):
        ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, 2, k, np.arange(trials), ztab)
        _compare(batch.trials_of(k), ref, np.arange(trials))
    batch.close()


def test_f4_cancel_reports_partial_results(gpu_lib):
    _say("f4 cancel, n=300")
    pim = gpu_lib
    n, R = 300, 64
    J, h = w.sk1(n, seed=2)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5)
    batch = pim.Batch([inst], R)
    T = 100000
    beta = np.full(T, 1.0)
    batch.run(beta, np.full(T, 0.4), seed=1, kernel="f4")
    batch.cancel()
    with pytest.raises(pim.PimError) as ei:
        batch.trials_of(0)
    assert ei.value.status == pim.PIM_ERR_CANCELLED
    batch.run(beta[:50], np.full(50, 0.4), seed=1, kernel="f4")
    batch.trials_of(0)


def test_f4_full_size_n1000_sampled(gpu_lib):
    """N = 1000 SK-1, 32 instances x 1024 trials x 400 steps: the launch the
    benchmark's large-N leg times.  Sampled trials of four instances are
    recomputed by the oracle in full; every trial's tracked best energy equals
    the Eq. (1) energy of its returned state."""
    _say("f4 n=1000 32x1024x400, sampled oracle trials")
    pim = gpu_lib
    n, R, T, count = 1000, 1024, 400, 32
    probs = [w.sk1(n, seed=3, index=k) for k in range(count)]
    ztab = w.gauss_table(8)
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, R).run(beta, eta, seed=8, kernel="f4")
    for k, trials in ((0, [0]), (9, [1023]), (17, [500]), (31, [127, 128])):
        J, h = probs[k]
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 8, k, trials, ztab)
        _compare(batch.trials_of(k), ref, trials)
    for k in range(0, count, 5):
        J, h = probs[k]
        got = batch.trials_of(k)
        S = got["best_state"].T.astype(np.int64)
        np.testing.assert_array_equal(pimi.energy_from_field(pimi.local_field(J, h, S), h, S), got["e_best"])
    batch.close()


@pytest.mark.parametrize("kernel", ["f4", "mfma"])
def test_f4_one_launch_for_all_parts(gpu_lib, kernel):
    """Several streamed parts of an uneven batch (e2m1 or int8 operands) run
    as one launch over a work list: partial trial blocks (200 trials), parts with and without fields,
    odd tile counts, and repeated runs that change the seed (the list is
    uploaded again) or keep it (reused); each result equals the oracle, and
    the third run equals the first."""
    _say(f"[{kernel}] f4 one launch over parts, 200 trials, fields")
    pim = gpu_lib
    ns = [300, 520, 300, 1000, 700, 130, 520]
    trials, steps = 200, 24
    ztab = w.gauss_table(8)
    probs = []
    for k, n in enumerate(ns):
        probs.append(_e2m1_instance(n, 17, k, (-2, -1, 0, 1, 2), hmax=3 if k % 3 == 1 else 0))
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, noise_table=ztab, rng_stream=40 + k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, trials)
    first = None
    for run, seed in enumerate((2, 5, 2)):
        batch.run(beta, eta, seed=seed, kernel=kernel)
        got = [batch.trials_of(k) for k in range(len(ns))]
        if run == 0:
            first = got
        if run < 2:
            for k, (J, h) in enumerate(probs):
                tr = np.arange(trials) if ns[k] <= 520 else np.array([0, 127, 128, 199])
                ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, seed, 40 + k, tr, ztab)
                _compare(got[k], ref, tr)
        else:
            for a, b in zip(first, got):
                for key in ("final", "e_best", "t_best", "best_state"):
                    np.testing.assert_array_equal(a[key], b[key])
    batch.close()


def test_f4_full_size_uneven_batch_sampled(gpu_lib):
    """The benchmark's uneven-N workload as it times it: 128 SK-1 instances,
    N_k = [100, 200, 400, 800, 1000][k mod 5], 1024 trials, here 2000 steps,
    one graph launch, e2m1 operands for N > 256 (one launch over all those
    parts), with first-hit targets.  Every trial equals the int8-operand run;
    sampled trials of six instances (every N) equal the oracle."""
    _say("f4 uneven N 128x1024x2000 graph, vs int8 and sampled oracle trials")
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
    batch.run(beta, eta, seed=2, target=tgt, kernel="mfma")
    i8 = [batch.trials_of(k) for k in range(count)]
    batch.run(beta, eta, seed=2, target=tgt, kernel="f4")
    for k in range(count):
        got = batch.trials_of(k)
        for key in ("final", "e_best", "t_best", "best_state", "first_hit", "e_final"):
            np.testing.assert_array_equal(got[key], i8[k][key], err_msg=f"instance {k} {key}")
    for k, trials in ((0, [0]), (1, [1023]), (2, [300]), (3, [511]), (4, [1000]), (122, [7])):
        J, h = probs[k]
        ref = _oracle(J, h, 1 / np.sqrt(ns[k]), beta, eta, 2, k, trials, ztab, target=tgt[k])
        _compare(batch.trials_of(k), ref, trials)
    batch.close()


@pytest.mark.parametrize("kernel", ["f4", "mfma"])
def test_f4_one_launch_cancel_and_target_toggle(gpu_lib, kernel):
    """The one launch over streamed parts (e2m1 or int8 operands): a run with
    first-hit targets, then the
    same schedule without them (the uploaded work list is reused, the target
    flag is a kernel argument), then a long run cancelled from the host, then
    a short run that completes; results equal the oracle where they are
    defined."""
    _say(f"[{kernel}] f4 one launch: targets on/off, cancel")
    pim = gpu_lib
    ns = [300, 600, 1000]
    trials, steps = 64, 30
    ztab = w.gauss_table(8)
    probs = [w.sk1(n, seed=23, index=k) for k, n in enumerate(ns)]
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, noise_table=ztab, rng_stream=60 + k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    tgt = [float(np.floor(-0.6 * n ** 1.5)) for n in ns]
    batch = pim.Batch(insts, trials)
    for use_target in (True, False):
        batch.run(beta, eta, seed=4, kernel=kernel, target=tgt if use_target else None)
        for k, (J, h) in enumerate(probs):
            got = batch.trials_of(k)
            ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, 4, 60 + k, np.arange(trials), ztab,
                          target=tgt[k] if use_target else None)
            _compare(got, ref, np.arange(trials))
            if not use_target:
                assert np.all(got["first_hit"] == -1)
    T = 60000
    batch.run(np.full(T, 1.0), np.full(T, 0.4), seed=1, kernel=kernel)
    batch.cancel()
    with pytest.raises(pim.PimError) as ei:
        batch.trials_of(0)
    assert ei.value.status == pim.PIM_ERR_CANCELLED
    batch.run(beta, eta, seed=4, kernel=kernel)
    for k, (J, h) in enumerate(probs):
        ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, 4, 60 + k, [0, 63], ztab)
        _compare(batch.trials_of(k), ref, [0, 63])
    batch.close()


LDS_CASES = [
    # n, trials, steps, values, hmax -- the LDS-resident e2m1 kernel (N <= 256)
    (1, 40, 30, (-1, 1), 0),
    (5, 64, 40, (-1, 0, 1), 2),
    (20, 64, 200, (-1, 1), 0),
    (31, 33, 60, (-2, -1, 1, 2), 0),         # last-tile tail of 12 registers
    (32, 64, 50, (-1, 1), 0),
    (33, 100, 40, (-6, -4, -3, -2, -1, 0, 1, 2, 3, 4, 6), 3),  # tail of 4, fields
    (64, 64, 40, (-1, 0, 1), 0),
    (100, 128, 40, (-1, 1), 0),
    (130, 70, 30, (-4, -2, 2, 4), 0),        # odd tile count: a padded half K step
    (200, 96, 50, (-1, 1), 0),               # tail of 8
    (224, 64, 30, (-3, 3), 5),
    (255, 32, 30, (-1, 1), 0),
    (256, 64, 24, (-1, 1), 1),
]


@pytest.mark.parametrize("case", LDS_CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}-{len(c[3])}v-h{c[4]}")
def test_f4_lds_parity(gpu_lib, case):
    n, trials, steps, values, hmax = case
    _say(f"f4 LDS kernel n={n} trials={trials} steps={steps} values={values} hmax={hmax}")
    probs = [_e2m1_instance(n, 41, k, values, hmax) for k in range(2)]
    batch, beta, eta, targets, ztab = _run(gpu_lib, probs, trials, steps, "f4", seed=15)
    for k, (J, h) in enumerate(probs):
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 15, 3 + k, np.arange(trials), ztab, target=targets[k])
        _compare(batch.trials_of(k), ref, np.arange(trials))
    batch.close()


def test_f4_lds_tuned_resume_and_recording(gpu_lib):
    """N = 200 with e2m1: after autotuning waves per workgroup, from caller
    spins, resumed in two halves; a recording run falls back to int8 and
    records the same trajectory."""
    _say("f4 LDS kernel: tuned, caller spins, resume, recording")
    pim = gpu_lib
    n, R, T = 200, 200, 120
    J, h = w.sk1(n, seed=8)
    ztab = w.gauss_table(8)
    inst = pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=5)
    beta = w.linear_beta(T)
    eta = w.eta_sqrt_beta_over_5(beta)
    init = np.random.default_rng(2).choice([-1, 1], size=(1, R, n)).astype(np.int8)
    b = pim.Batch([inst], R, init_spins=init)
    b.tune(steps=50)
    full = b.run(beta, eta, seed=3, kernel="f4").trials_of(0)
    ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 3, 5, [0, 127, 128, 199], ztab,
                  init=init[0][[0, 127, 128, 199]].T.astype(np.int64))
    _compare(full, ref, [0, 127, 128, 199])
    a1 = pim.Batch([inst], R, init_spins=init).run(beta[:60], eta[:60], seed=3, kernel="f4").trials_of(0)
    a2 = pim.Batch([inst], R, init_spins=a1["final"][None]).run(beta[60:], eta[60:], seed=3, start_step=60,
                                                               kernel="f4").trials_of(0)
    np.testing.assert_array_equal(a2["final"], full["final"])
    np.testing.assert_array_equal(np.minimum(a1["e_best"], a2["e_best"]), full["e_best"])
    rec = pim.Batch([inst], 32, init_spins=init[:, :32]).run(beta[:20], eta[:20], seed=3, kernel="f4", record=True)
    rec8 = pim.Batch([inst], 32, init_spins=init[:, :32]).run(beta[:20], eta[:20], seed=3, kernel="mfma", record=True)
    np.testing.assert_array_equal(rec.states(0, 7), rec8.states(0, 7))


def test_f4_lds_full_size_sk200_equals_int8(gpu_lib):
    """The headline workload, 128 SK-1 N = 200 instances x 1024 trials x 10^4
    steps with first-hit targets, on e2m1 operands: every trial equals the
    int8 kernel's run, and sampled trials equal the oracle."""
    _say("f4 LDS kernel sk200 128x1024x10000 vs int8, sampled oracle trials")
    pim = gpu_lib
    n, R, T, I = 200, 1024, 10000, 128
    ztab = w.gauss_table(8)
    probs = [w.sk1(n, seed=1, index=k) for k in range(I)]
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(n), xi=0.5, noise_table=ztab, rng_stream=k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    tgt = [-2000.0] * I
    batch = pim.Batch(insts, R)
    batch.run(beta, eta, seed=1, target=tgt, kernel="mfma")
    i8 = [batch.trials_of(k) for k in range(I)]
    batch.run(beta, eta, seed=1, target=tgt, kernel="f4")
    for k in range(I):
        got = batch.trials_of(k)
        for key in ("final", "e_best", "t_best", "best_state", "first_hit", "e_final"):
            np.testing.assert_array_equal(got[key], i8[k][key], err_msg=f"instance {k} {key}")
    for k, trials in ((0, [0]), (77, [1023])):
        J, h = probs[k]
        ref = _oracle(J, h, 1 / np.sqrt(n), beta, eta, 1, k, trials, ztab, target=tgt[k])
        _compare(batch.trials_of(k), ref, trials)
    batch.close()


@pytest.mark.parametrize("kernel", ["f4", "mfma"])
def test_f4_one_launch_caller_initial_spins(gpu_lib, kernel):
    """The one launch over streamed parts (e2m1 or int8 operands) starting
    from caller spins (each part's own initial-state buffer travels in the
    launch's part table)."""
    _say(f"[{kernel}] f4 one launch from caller spins")
    pim = gpu_lib
    ns = [400, 700, 300]
    trials, steps = 48, 20
    ztab = w.gauss_table(8)
    probs = [w.sk1(n, seed=29, index=k) for k, n in enumerate(ns)]
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, noise_table=ztab, rng_stream=80 + k)
             for k, (J, h) in enumerate(probs)]
    rng = np.random.default_rng(5)
    init = [rng.choice([-1, 1], size=(trials, n)).astype(np.int8) for n in ns]
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, trials, init_spins=init).run(beta, eta, seed=6, kernel=kernel)
    for k, (J, h) in enumerate(probs):
        tr = [0, 17, 47]
        ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, 6, 80 + k, tr, ztab, init=init[k][tr].T.astype(np.int64))
        _compare(batch.trials_of(k), ref, tr)
    batch.close()


@pytest.mark.parametrize("exact", [(0, 1), (0,)])
def test_one_launch_with_parts_on_both_operand_types(gpu_lib, exact):
    """e2m1 operands asked for, but only the parts listed in `exact` have
    e2m1-exact couplings; the others (couplings of 5 and 7) fall back to int8.
    With two exact parts they run as the one e2m1 launch and the int8 parts as
    their own launches; with one, the int8 parts run as the one launch and the
    e2m1 part alone.  Sampled trials of every part equal the oracle."""
    _say(f"one launch, parts on both operand types, exact parts {exact}")
    pim = gpu_lib
    ns = [300, 600, 400, 700, 100]
    trials, steps = 160, 24
    ztab = w.gauss_table(8)
    probs = [_e2m1_instance(n, 41, k, (-2, -1, 0, 1, 2) if k in exact or n <= 256 else (-7, -5, -1, 1, 5, 7))
             for k, n in enumerate(ns)]
    insts = [pim.Instance(J, h, j_scale=1 / np.sqrt(len(h)), xi=0.5, noise_table=ztab, rng_stream=90 + k)
             for k, (J, h) in enumerate(probs)]
    beta = w.linear_beta(steps, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    batch = pim.Batch(insts, trials).run(beta, eta, seed=8, kernel="f4")
    for k, (J, h) in enumerate(probs):
        tr = [0, 127, 128, 159]
        ref = _oracle(J, h, 1 / np.sqrt(len(h)), beta, eta, 8, 90 + k, tr, ztab)
        _compare(batch.trials_of(k), ref, tr)
    batch.close()
