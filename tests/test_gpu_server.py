"""GPU tests of the request server (continuous batching): results equal the
batch API's for the same request (same rule, seed and noise stream = id),
are the same alone and in a mixed stream, and admission honours the slot
table and the device-memory budget."""
import time

import numpy as np
import pytest

import workloads as w
from oracle import pimi

pytestmark = pytest.mark.gpu

STEPS = 32
BETA = w.constant(STEPS, 1.0)
ETA = w.mimo_eta(STEPS, 0.05, 0.3)


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _request(pim, k, nt, qam):
    p = w.mimo.mimo_problem(nt, nt, qam, 15.0, seed=4, index=k)
    return pim.mimo_ising(p["H"], p["y"], qam, "di", p["esn0"])[:2]


def _drain(srv, want, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        ids, st, e = srv.poll()
        for i, s, x in zip(ids, st, e):
            got[int(i)] = (s.copy(), float(x))
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(got)} of {want} requests finished")
    return got


def _server(pim, **kw):
    args = dict(max_n=128, trials=32, beta=BETA, eta=ETA, xi=2.0, noise_table=w.gauss_table(8), prec="fp8",
                slots_per_class=256, max_batch=32, streams=3, seed=7)
    args.update(kw)
    return pim.Server(**args)


def test_server_matches_batch_api_and_alone_equals_mix(gpu_lib):
    _say("server: batch-API equality, alone vs mix")
    pim = gpu_lib
    J, h = _request(pim, 0, 8, 16)
    n = J.shape[0]
    # batch API reference: same rule, seed, stream = request id
    inst = pim.Instance(J, h, j_scale=1.0, xi=2.0, noise_table=w.gauss_table(8), rng_stream=777, prec="fp8")
    b = pim.Batch([inst], 32).run(BETA, ETA, seed=7)
    ref_s, ref_e, _, _ = b.best(0)
    b.close()
    srv = _server(pim)
    assert srv.submit([777], [J], [h]) == 1
    assert srv.flush() == 1
    alone = _drain(srv, 1)[777]
    assert np.array_equal(alone[0][:n], ref_s) and alone[1] == ref_e
    # the same request among 150 others of mixed sizes, submitted in waves
    shapes = [(8, 4), (16, 16), (4, 16), (32, 4), (8, 16)]
    reqs = [(5000 + k, *_request(pim, k + 1, *shapes[k % len(shapes)])) for k in range(150)]
    reqs.insert(77, (777, J, h))
    for start in range(0, len(reqs), 40):
        part = reqs[start:start + 40]
        left = part
        while left:
            took = srv.submit([r[0] for r in left], [r[1] for r in left], [r[2] for r in left])
            srv.flush()
            left = left[took:]
            if left:
                time.sleep(0.001)
    got = _drain(srv, len(reqs) - 0)
    assert set(got) == {r[0] for r in reqs}
    assert np.array_equal(got[777][0][:n], alone[0][:n]) and got[777][1] == alone[1]
    srv.close()
    # every request of the mix equals the same request through the batch API
    # (rng stream = id; instances of different N run as one uneven batch), and
    # its reported energy is the oracle's binary64 Eq. (1) energy of its state
    insts = [pim.Instance(J_, h_, j_scale=1.0, xi=2.0, noise_table=w.gauss_table(8), rng_stream=rid, prec="fp8")
             for rid, J_, h_ in reqs]
    b = pim.Batch(insts, 32).run(BETA, ETA, seed=7)
    for k, (rid, J_, h_) in enumerate(reqs):
        m = J_.shape[0]
        s_ref, e_ref, _, _ = b.best(k)
        assert np.array_equal(got[rid][0][:m], s_ref) and got[rid][1] == e_ref, rid
        assert got[rid][1] == pytest.approx(pimi.energy_f64(J_, h_, got[rid][0][:m].astype(np.float64)),
                                            rel=1e-9, abs=1e-9), rid
    b.close()


def _dyadic_fp8(n, seed):
    """Couplings whose FP8 quantisation on the device is exact (q in e4m3,
    max |q| = 448 so the scale is 2^-6) and fields on the same grid: every
    binary32 operation of the sweep is exact."""
    rng = np.random.default_rng([seed, n])
    q = np.triu(rng.integers(-16, 17, size=(n, n)).astype(np.float64), 1)
    q = q + q.T
    q[0, 1] = q[1, 0] = 448.0
    return q * 2.0 ** -6, rng.integers(-1000, 1001, size=n) * 2.0 ** -6


def test_server_dyadic_requests_bit_exact_vs_oracle(gpu_lib):
    """Requests through pim_server_* (binary64 staging, device-side FP8
    quantisation, chunked sweep, binary64 re-rank and selection) against the
    binary64 oracle: the returned state is the oracle's best trial state (ties
    to the lowest trial) and the energy is its Eq. (1) energy, exactly."""
    _say("server: dyadic requests vs the oracle")
    pim = gpu_lib
    # small chunks of mixed classes (the latency form of the sweep), then one
    # chunk of 160 requests of one class (more than 128 trial blocks: the
    # batched form)
    sizes = [16, 40, 64, 100, 128, 33, 64, 96]
    small = [(300 + k, *_dyadic_fp8(sizes[k % len(sizes)], seed=k)) for k in range(24)]
    large = [(400 + k, *_dyadic_fp8(64, seed=100 + k)) for k in range(160)]
    got = {}
    for reqs, max_batch, slots in ((small, 8, 64), (large, 160, 160)):
        srv = _server(pim, max_n=128, max_batch=max_batch, slots_per_class=slots)
        left = reqs
        took = srv.submit([r[0] for r in left], [r[1] for r in left], [r[2] for r in left])
        assert took == len(reqs)
        srv.flush()
        got.update(_drain(srv, len(reqs)))
        srv.close()
    reqs = small + large
    ztab = w.gauss_table(8)
    for rid, J, h in reqs:
        n = J.shape[0]
        ref = pimi.run_parallel(pimi.RealProblem(J, h, 1.0, 2.0, 4, ztab), BETA, ETA, 7, rid, np.arange(32))
        e_all = pimi.energy_f64(J, h, ref["best_state"].astype(np.float64))
        a = int(np.argmin(e_all))
        assert np.array_equal(got[rid][0][:n], ref["best_state"][:, a].astype(np.int8)), rid
        assert got[rid][1] == float(e_all[a]), rid


def test_server_admission_limits(gpu_lib):
    _say("server: admission by slots and budget")
    pim = gpu_lib
    J, h = _request(pim, 3, 8, 4)  # N = 32
    srv = _server(pim, slots_per_class=8, max_batch=8)
    ids = list(range(20))
    assert srv.submit(ids, [J] * 20, [h] * 20) == 8     # one chunk of 8 slots
    assert srv.pending() == (8, 0)
    assert srv.flush() == 8
    assert srv.submit(ids[8:], [J] * 12, [h] * 12) == 0  # the only chunk is in flight
    got = _drain(srv, 8)
    assert set(got) == set(range(8))
    assert srv.submit(ids[8:], [J] * 12, [h] * 12) == 8  # the chunk is free again
    srv.flush()
    _drain(srv, 8)
    srv.close()
    tiny = _server(pim, hbm_budget=1024)
    assert tiny.submit([1], [J], [h]) == 0               # a chunk needs more than the budget
    tiny.close()


def test_server_parallel_staging_and_rejection(gpu_lib):
    """Large submissions are validated and staged by the server's host workers:
    their results equal the same requests submitted one at a time.  An
    invalid request is rejected; the requests before it are admitted, counted
    in the error, and finish normally."""
    _say("server: parallel staging, rejection with partial admission")
    pim = gpu_lib
    shapes = [(64, 16), (32, 16), (8, 4), (64, 4), (16, 16)]   # N = 256, 128, 16, 128, 64
    reqs = [(900 + k, *_request(pim, 40 + k, *shapes[k % len(shapes)])) for k in range(12)]
    one = _server(pim, max_n=256)
    for rid, J, h in reqs:                      # one at a time: the calling thread alone
        assert one.submit([rid], [J], [h]) == 1
        one.flush()
    ref = _drain(one, len(reqs))
    one.close()
    many = _server(pim, max_n=256)
    assert many.submit([r[0] for r in reqs], [r[1] for r in reqs], [r[2] for r in reqs]) == len(reqs)
    many.flush()
    got = _drain(many, len(reqs))
    for rid, J, _ in reqs:
        n = J.shape[0]
        assert np.array_equal(got[rid][0][:n], ref[rid][0][:n]) and got[rid][1] == ref[rid][1], rid
    # rejection: the third request is not symmetric
    J0, h0 = reqs[0][1], reqs[0][2]
    bad = J0.copy()
    bad[3, 5] += 1e-9
    with pytest.raises(pim.PimError) as ei:
        many.submit([1, 2, 3, 4], [J0, reqs[1][1], bad, J0], [h0, reqs[1][2], h0, h0])
    assert ei.value.admitted == 2 and "symmetric" in str(ei.value)
    assert many.pending() == (2, 0)
    many.flush()
    assert set(_drain(many, 2)) == {1, 2}
    many.close()


MIMO_SHAPES = [(8, 8, 4, "di"), (8, 8, 16, "di"), (16, 16, 16, "di"), (16, 16, 4, "ml"), (12, 8, 16, "di"),
               (32, 32, 4, "di"), (8, 6, 16, "ml"), (64, 64, 16, "di"), (16, 12, 4, "di"), (64, 64, 4, "ml")]


def test_server_batching_wait_only_while_class_in_flight(gpu_lib):
    """pim_server_flush launches a partly filled chunk at once when no chunk
    of its class is in flight, and holds it (up to max_wait_us) while one is."""
    _say("server: batching wait only under load")
    pim = gpu_lib
    J, h = _request(pim, 5, 8, 4)  # N = 32
    J2, h2 = _request(pim, 6, 16, 4)  # N = 64, another class
    srv = _server(pim, max_wait_us=1e9, slots_per_class=64, max_batch=8)
    assert srv.submit([1], [J], [h]) == 1
    assert srv.flush() == 1                  # idle class: launched at once
    assert srv.submit([2, 3], [J, J], [h, h]) == 2
    assert srv.flush() == 0                  # its class has a chunk in flight: held
    assert srv.submit([4], [J2], [h2]) == 1
    assert srv.flush() == 1                  # an idle class is not held by another
    got = _drain(srv, 2)                     # collecting request 1 makes its class idle
    assert set(got) == {1, 4}
    assert srv.flush() == 2
    assert set(_drain(srv, 2)) == {2, 3}
    srv.close()


def _mimo_problem(k, nr, nt, qam, db=15.0):
    return w.mimo.mimo_problem(nt, nr, qam, db, seed=12, index=k)


def test_device_mimo_mapping_matches_host_and_oracle(gpu_lib):
    """The server's device mapping kernel (binary64 Gram, LDL^T MMSE solve,
    slicing, J and h) against the host library's mapping (same operation
    order: identical) and the oracle's (Suppl. "Delta-Ising MIMO"; 1e-12)."""
    from oracle import mimo
    pim = gpu_lib
    for k, (nr, nt, qam, mapping) in enumerate(MIMO_SHAPES * 2):
        _say(f"device MIMO mapping nr={nr} nt={nt} qam={qam} {mapping}")
        p = _mimo_problem(k, nr, nt, qam)
        Jd, hd, xd = pim.mimo_ising_device(p["H"], p["y"], qam, mapping, p["esn0"])
        Jh, hh, xh = pim.mimo_ising(p["H"], p["y"], qam, mapping, p["esn0"])
        d = mimo.detector_instance(p, mapping)
        assert np.array_equal(xd, d["xm"]) and np.array_equal(xd, xh)
        scale = np.abs(d["J"]).max()
        np.testing.assert_allclose(Jd, d["J"], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(hd, d["h"], rtol=0, atol=1e-12 * max(np.abs(d["h"]).max(), 1.0))
        print(f"  host identical: J {np.array_equal(Jd, Jh)} h {np.array_equal(hd, hh)}", flush=True)


def test_device_mimo_mapping_singular_systems_agree_with_host(gpu_lib):
    """Numerically singular MMSE systems (equal or proportional channel
    columns, a regulariser 1/(Es/N0) below rounding): host and device take the
    same LDL^T steps, so both reject the system (a pivot that is not
    positive) or both return the same mapping bit for bit."""
    pim = gpu_lib
    rng = np.random.default_rng(5)

    def outcome(fn, H, y, esn0):
        try:
            return True, fn(H, y, 16, "di", esn0)
        except pim.PimError as e:
            assert "positive definite" in str(e), e
            return False, None

    cases = [(np.ones((2, 2), complex), 1e300), (np.ones((2, 2), complex), 10.0)]
    for k in range(6):
        nt = 2 + 3 * k
        H = (rng.standard_normal((nt + 1, nt)) + 1j * rng.standard_normal((nt + 1, nt))) / np.sqrt(2)
        H[:, -1] = (k + 1) * H[:, 0]
        cases.append((H, 1e300))
    accepted = []
    for i, (H, esn0) in enumerate(cases):
        y = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
        _say(f"singular MMSE case {i}: nr={H.shape[0]} nt={H.shape[1]} esn0={esn0:g}")
        ok_h, rh = outcome(pim.mimo_ising, H, y, esn0)
        ok_d, rd = outcome(pim.mimo_ising_device, H, y, esn0)
        assert ok_h == ok_d, (i, ok_h, ok_d)
        if ok_h:
            for a, b in zip(rh, rd):
                assert np.array_equal(a, b), i
        accepted.append(ok_h)
    # two equal columns, regulariser below rounding: the second pivot is exactly 0
    assert accepted[0] is False and accepted[1] is True


def test_mimo_server_matches_host_staged_server(gpu_lib):
    """The same detection problems through the MIMO server ((H, y) staged,
    Ising instance built on the device) and through the (J, h) server (host
    mapping): the same states, binary64 energies within 1e-12 (equal when the
    two mappings are bit-identical), x_m equal; every energy equals the
    oracle's Eq. (1) energy of the returned state on the oracle's own
    instance within 1e-9 (P14)."""
    from oracle import mimo
    pim = gpu_lib
    reqs = []
    for k in range(60):
        nr, nt, qam, mapping = MIMO_SHAPES[k % len(MIMO_SHAPES)]
        reqs.append((2000 + k, nr, nt, qam, mapping, _mimo_problem(100 + k, nr, nt, qam)))
    kw = dict(max_n=256, max_batch=16, slots_per_class=64)
    dev = _server(pim, mimo=True, **kw)
    host = _server(pim, **kw)
    _say("MIMO server: device mapping vs host-staged requests")
    assert dev.submit_mimo([r[0] for r in reqs], [r[5]["H"] for r in reqs], [r[5]["y"] for r in reqs],
                           [r[3] for r in reqs], [r[4] for r in reqs], [r[5]["esn0"] for r in reqs]) == len(reqs)
    dev.flush()
    maps = [pim.mimo_ising(r[5]["H"], r[5]["y"], r[3], r[4], r[5]["esn0"]) for r in reqs]
    assert host.submit([r[0] for r in reqs], [m[0] for m in maps], [m[1] for m in maps]) == len(reqs)
    host.flush()
    got_d, xms = {}, {}
    t0 = time.time()
    while len(got_d) < len(reqs):
        ids, st, e, xm, tm = dev.poll_mimo()
        for i, sv, ev, xv, tv in zip(ids, st, e, xm, tm):
            got_d[int(i)] = (sv.copy(), float(ev))
            xms[int(i)] = xv.copy()
            assert tv[0] <= tv[1] <= tv[2]
        assert time.time() - t0 < 60
    got_h = _drain(host, len(reqs))
    dev.close()
    host.close()
    for (rid, nr, nt, qam, mapping, p), (J, h, xm) in zip(reqs, maps):
        n = J.shape[0]
        assert np.array_equal(xms[rid][:2 * nt], xm) and not xms[rid][2 * nt:].any(), rid
        assert np.array_equal(got_d[rid][0][:n], got_h[rid][0][:n]), rid
        assert got_d[rid][1] == pytest.approx(got_h[rid][1], rel=1e-12, abs=1e-9), rid
        d = mimo.detector_instance(p, mapping)
        e_orc = pimi.energy_f64(d["J"], d["h"], got_d[rid][0][:n].astype(np.float64))
        assert got_d[rid][1] == pytest.approx(e_orc, rel=1e-9, abs=1e-9), rid
        x = pim.mimo_decode(xms[rid][:2 * nt], got_d[rid][0][:n], qam, mapping)
        assert np.array_equal(x, mimo.decode(d["xm"], d["T"], got_d[rid][0][:n], qam)), rid


def test_mimo_server_rejects_invalid_requests(gpu_lib):
    pim = gpu_lib
    _say("MIMO server: validation")
    srv = _server(pim, mimo=True, max_n=64)
    p = _mimo_problem(1, 8, 8, 16)
    J, h = pim.mimo_ising(p["H"], p["y"], 16, "di", p["esn0"])[:2]
    with pytest.raises(pim.PimError) as ei:
        srv.submit([1], [J], [h])
    assert ei.value.status == pim.PIM_ERR_STATE
    bad_H = p["H"].copy()
    bad_H[2, 3] = np.nan
    with pytest.raises(pim.PimError) as ei:
        srv.submit_mimo([1, 2, 3], [p["H"], p["H"], bad_H], [p["y"]] * 3, 16, "di", p["esn0"])
    assert ei.value.admitted == 2 and "finite" in str(ei.value)
    big = _mimo_problem(2, 32, 32, 16)  # N = 128 > max_n
    with pytest.raises(pim.PimError) as ei:
        srv.submit_mimo([4], [big["H"]], [big["y"]], 16, "di", big["esn0"])
    assert ei.value.admitted == 0
    assert srv.pending() == (2, 0)
    srv.flush()
    assert set(_drain(srv, 2)) == {1, 2}
    srv.close()
