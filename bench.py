"""Benchmark: batched PIMI sweep on SK-1 N=200 on one MI355X.

One step = the whole hot path over one batch whose inputs are resident on
the device: the persistent int8-MFMA sweep of every trial of every instance,
the binary64 re-rank of every trial's best state, and the per-instance argmin
readout.  The instances are staged in device memory before the timed region,
and the per-step threshold tables are compiled and uploaded by the warm-up
(the timed steps run the same schedule, so the library reuses them).
The same timed protocol then runs on e2m1 (FP4) operands ("e2m1" in the
line): the couplings and spins are exact e2m1 values, so its results must
equal the int8 run's, which the line records.

Success for TTS99 (Sec. III.A, Eqs. (5)-(6)) is measured against a reference
energy per instance: the lower of the simulated-annealing reference (the
paper's SK-1 ground-truth recipe, stored in tests/golden/sa_ref.json by a
script that runs only the CPU oracle) and the best energy of the warm-up runs.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Workload defaults: 128 SK-1 instances of N = 200
(J = +-1, h = 0), 1024 trials each, 10^4 synchronous steps, beta linear
0.1 -> 3.0, eta = sqrt(beta / 5), xi = 0.5, c = 1/sqrt(N), 4-level LUT, 8-bit
Gaussian noise.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The request server runs up to 16 streams; the HIP runtime maps streams onto
# this many hardware queues (its default is 4), read once when it starts, so
# it is set before torch loads.  The other legs use one or two streams.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

INT8_MFMA_PEAK = 5.0e15            # dense int8 MFMA, ops/s (MI355X)
FP4_MFMA_PEAK = 10.1e15           # dense FP4 (e2m1) MFMA, ops/s (MI355X)
# 32-bit VALU lane-ops/s: CUs x SIMDs x 32 lanes per clock x clock, i.e. the published FP32 vector
# rate (157.3 TFLOP/s) with a fused multiply-add counted as one lane-op
VALU_PEAK = 256 * 4 * 32 * 2.4e9
HBM_PEAK = 8.0e12
LDS_PEAK = 256 * 256 * 2.4e9       # LDS read bytes/s: CUs x 256 B/clk (128-bit reads) x clock


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=128)
    ap.add_argument("--trials", type=int, default=1024)
    ap.add_argument("--sweeps", type=int, default=10000, help="update steps T per trial")
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--kernel", default="mfma", choices=["mfma", "plain", "f4"],
                    help="mfma: int8 operands; f4: e2m1 (FP4) operands (exact for J = +-1, identical results)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-trials", type=int, default=512)
    ap.add_argument("--cpu-steps", type=int, default=2000)
    ap.add_argument("--plain-instances", type=int, default=8,
                    help="instances run through the plain FP32 per-instance kernel for the comparison "
                         "(0 = skip); trajectories are bit-identical, so TTS99 is equal")
    ap.add_argument("--core-only", action="store_true",
                    help="only the SK-1 N=200 sweep (no plain, MIMO, serving, uneven-N, comparison or CPU legs)")
    ap.add_argument("--no-mimo", action="store_true", help="skip the MIMO detection leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-N batched leg")
    ap.add_argument("--no-mimo-grid", action="store_true", help="skip the MIMO detection grid")
    ap.add_argument("--grid-channels", type=int, default=256, help="channels per MIMO grid point")
    ap.add_argument("--no-serving", action="store_true", help="skip the MIMO serving leg")
    ap.add_argument("--serving-mix", default="both", choices=["5g", "full", "both"])
    ap.add_argument("--serving-streams", type=int, default=16)
    ap.add_argument("--serving-batch", type=int, default=0, help="requests per launch (0: 256 for the 5G mix, "
                    "64 for the full mix)")
    ap.add_argument("--serving-prealloc", type=int, default=0, help="chunks allocated up front per size class "
                    "(0: 16)")
    ap.add_argument("--serving-requests", type=int, default=100000,
                    help="requests per arrival rate (the paper's throughput protocol uses 10^5)")
    ap.add_argument("--uneven-steps", type=int, default=10000, help="steps of the uneven-N batched leg")
    ap.add_argument("--no-tts-scan", action="store_true", help="skip the TTS99 scan over the anneal length")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the parallel-vs-sequential comparison and the flip-rate diagnostic")
    ap.add_argument("--mimo-requests", type=int, default=512,
                    help="MIMO channels in the batched quality/throughput run")
    ap.add_argument("--mimo-latency", type=int, default=200,
                    help="single requests timed per kernel for the latency percentiles")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes (x3), for calibrating the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count")
    return ap.parse_args()


def copy_probe(nbytes):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}), flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden")


def sa_reference(name, n, seed, count):
    """Simulated-annealing reference energies of workloads.sk1(n, seed, k),
    k < count, from the stored set `name`, or None when the set does not
    cover them all."""
    path = os.path.join(GOLDEN, "sa_ref.json")
    if not os.path.exists(path):
        return None
    rows = {(r["n"], r["seed"], r["index"]): r["e_sa"] for r in json.load(open(path)).get(name, [])}
    got = [rows.get((n, seed, k)) for k in range(count)]
    return None if any(v is None for v in got) else got


def sa_reference_uneven(ns, seed):
    path = os.path.join(GOLDEN, "sa_ref.json")
    if not os.path.exists(path):
        return None
    rows = {(r["n"], r["seed"], r["index"]): r["e_sa"] for r in json.load(open(path)).get("uneven", [])}
    got = [rows.get((n, seed, k)) for k, n in enumerate(ns)]
    return None if any(v is None for v in got) else got


def n99_of(p):
    """Eq. (5) with epsilon = 0.01: independent trials for 99 % success."""
    return 1 if p >= 1 else (None if p <= 0 else math.ceil(math.log(0.01) / math.log(1 - p)))


def reference_summary(gpu_best, e_sa):
    """How the GPU's best energies compare with the annealing reference."""
    g = np.asarray(gpu_best, dtype=np.float64)
    a = np.asarray(e_sa, dtype=np.float64)
    d = g - a
    return {"instances": len(g), "gpu_below_sa": int((d < 0).sum()), "gpu_equal_sa": int((d == 0).sum()),
            "gpu_above_sa": int((d > 0).sum()),
            "gap_gpu_minus_sa": {"mean": float(d.mean()), "min": float(d.min()), "max": float(d.max())},
            "rel_gap_mean": float((d / np.abs(a)).mean())}


def measured_traffic():
    """HBM bytes per launch of the sweep kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sweep_mfma_sk200_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith(" "))
    csrc = os.path.join(ROOT, "paper_2604_17109_amd", "csrc")
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                  for f in ["sweep_mfma.hip", "philox.hpp", "internal.hpp"])).hexdigest()[:16]
    if kv.get("kernel_source_sha256_16") != sha:
        return None
    return int(kv["hbm_bytes_per_launch"])


def cpu_baseline(n, trials, steps, xi, c):
    """The oracle as it stands, on one SK-1 instance: `trials` trials for the
    first `steps` steps of the same schedule (per-step cost is constant)."""
    import workloads as w
    from oracle import pimi
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count() or 1
    J, h = w.sk1(n, seed=1, index=0)
    beta = w.linear_beta(10000)[:steps]
    eta = w.eta_sqrt_beta_over_5(beta)
    prob = pimi.Problem(J, h, c=c, xi=xi, levels=4, ztab=w.gauss_table(8))
    t0 = time.perf_counter()
    pimi.run_parallel(prob, beta, eta, 1, 0, np.arange(trials))
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": trials * steps * n / dt, "unit": "spin-updates/s", "cores": int(threads),
            "kind": "oracle", "cpu_model": model, "nproc": os.cpu_count(),
            "sample": f"SK-1 N={n} instance 0, {trials} trials x first {steps} of the 10^4 steps "
                      f"({dt:.1f} s, NumPy binary64 on the host)"}


MIMO = {"nt": 16, "nr": 16, "qam": 16, "ebn0_db": 20.0, "mapping": "di", "trials": 32, "steps": 64,
        "gamma": (0.05, 0.3), "xi": 2.0, "beta": 1.0}


def mimo_leg(args):
    """MIMO detection (Suppl. "PIMI FPGA implementation for MIMO detection"):
    16x16 16-QAM at Eb/N0 = 20 dB, DI mapping (64 spins), 32 trials x 64 steps,
    beta = 1, xi = 2, eta = sqrt(1 / (5 gamma(t))) with gamma 0.05 -> 0.3.

    * latency: one request at a time (instance upload, sweep, binary64
      re-rank, readback of the detected state), p50 / p99 over requests, for
      the FP8 and BF16 MFMA kernels and the plain FP32 kernel; the sweep kernel's
      own duration (HIP events) alongside;
    * quality and throughput: all requests in one batch (one launch), symbol
      and bit error rates against the transmitted symbols and the sliced MMSE
      estimate the mapping starts from."""
    import torch
    import paper_2604_17109_amd as pim
    import workloads as w
    cfg = MIMO
    T, R, qam, nt = cfg["steps"], cfg["trials"], cfg["qam"], cfg["nt"]
    beta = w.constant(T, cfg["beta"])
    eta = w.mimo_eta(T, *cfg["gamma"])
    ztab = w.gauss_table(8)
    M = args.mimo_requests
    probs = [w.mimo.mimo_problem(nt, cfg["nr"], qam, cfg["ebn0_db"], seed=7, index=k) for k in range(M)]
    maps = [pim.mimo_ising(p["H"], p["y"], qam, cfg["mapping"], p["esn0"]) for p in probs]
    n = maps[0][0].shape[0]
    out = {"workload": f"{nt}x{cfg['nr']} {qam}-QAM, Eb/N0 {cfg['ebn0_db']} dB, {cfg['mapping'].upper()} mapping, "
                       f"N = {n} spins, {R} trials x {T} steps",
           "requests": M}

    def one_request(k, prec, kernel):
        J, h, xm = maps[k]
        t0 = time.perf_counter()
        inst = pim.Instance(J, h, j_scale=1.0, xi=cfg["xi"], levels=4, noise_table=ztab, rng_stream=k, prec=prec)
        b = pim.Batch([inst], R)
        b.run(beta, eta, seed=11, kernel=kernel)
        spins, e, _, _ = b.best(0)
        dt = time.perf_counter() - t0
        kms = b.kernel_ms()
        b.close()
        inst.close()
        return dt * 1e6, kms * 1e3, pim.mimo_decode(xm, spins, qam, cfg["mapping"])

    lat = {}
    for name, prec, kernel in (("fp8_mfma", "fp8", "mfma"), ("bf16_mfma", "bf16", "mfma"),
                               ("plain_f32", "fp8", "plain")):
        for k in range(5):
            one_request(k, prec, kernel)  # warm-up
        e2e, kus = [], []
        for k in range(min(args.mimo_latency, M)):
            a, b_, _ = one_request(k, prec, kernel)
            e2e.append(a)
            kus.append(b_)
        lat[name] = {"e2e_p50_us": float(np.percentile(e2e, 50)), "e2e_p99_us": float(np.percentile(e2e, 99)),
                     "kernel_p50_us": float(np.percentile(kus, 50)), "kernel_p99_us": float(np.percentile(kus, 99))}
    # the same requests one at a time through the request server (FP8), which
    # keeps its device buffers and step tables between requests: submit ->
    # launch at once (no batching wait) -> poll until the result is readable
    srv = pim.Server(max_n=n, trials=R, beta=beta, eta=eta, xi=cfg["xi"], noise_table=ztab, prec="fp8",
                     slots_per_class=4, max_batch=1, streams=1, seed=11, max_wait_us=0.0, prealloc_chunks=1)
    e2e, same = [], 0
    for k in range(-5, min(args.mimo_latency, M)):  # the first 5 are a warm-up
        kk = max(k, 0)
        J, h, xm = maps[kk]
        t0 = time.perf_counter()
        srv.submit([kk], [J], [h])
        srv.flush()
        got = []
        while not len(got):
            got, st, _ = srv.poll()
        dt = time.perf_counter() - t0
        if k >= 0:
            e2e.append(dt * 1e6)
            x = pim.mimo_decode(xm, st[0][:n], qam, cfg["mapping"])
            same += int(np.array_equal(x, one_request(kk, "fp8", "mfma")[2]))
    srv.close()
    lat["server_fp8"] = {"e2e_p50_us": float(np.percentile(e2e, 50)), "e2e_p99_us": float(np.percentile(e2e, 99)),
                         "same_detection_as_one_shot": same / len(e2e)}
    lat["kernel_p99_speedup_fp8_vs_plain"] = lat["plain_f32"]["kernel_p99_us"] / lat["fp8_mfma"]["kernel_p99_us"]
    lat["e2e_p99_speedup_fp8_vs_plain"] = lat["plain_f32"]["e2e_p99_us"] / lat["fp8_mfma"]["e2e_p99_us"]
    out["latency"] = lat

    # batched: all requests in one launch
    bits_per_sym = w.mimo.bits_per_symbol(qam)
    quality = {}
    for name, prec in (("fp8_mfma", "fp8"), ("bf16_mfma", "bf16")):
        insts = [pim.Instance(J, h, j_scale=1.0, xi=cfg["xi"], levels=4, noise_table=ztab, rng_stream=k, prec=prec)
                 for k, (J, h, xm) in enumerate(maps)]
        b = pim.Batch(insts, R)
        b.run(beta, eta, seed=11)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(beta, eta, seed=11)
        dets = [b.best(k)[0] for k in range(M)]
        dt = time.perf_counter() - t0
        kms = b.kernel_ms()
        se = be = 0
        for k, p in enumerate(probs):
            x = pim.mimo_decode(maps[k][2], dets[k], qam, cfg["mapping"])
            se += int(np.count_nonzero(x != p["x"]))
            be += int(np.count_nonzero(w.mimo.bits_from_symbols(x, qam) != p["bits"]))
        quality[name] = {"ser": se / (M * nt), "ber": be / (M * nt * bits_per_sym),
                         "requests_per_s": M / dt, "kernel_ms": kms,
                         "spin_updates_per_s": M * R * T * n / (kms / 1e3)}
        b.close()
        for i in insts:
            i.close()
    se = be = 0
    for k, p in enumerate(probs):
        xm = maps[k][2]
        x = xm[:nt] + 1j * xm[nt:]
        se += int(np.count_nonzero(x != p["x"]))
        be += int(np.count_nonzero(w.mimo.bits_from_symbols(x, qam) != p["bits"]))
    quality["mmse"] = {"ser": se / (M * nt), "ber": be / (M * nt * bits_per_sym)}
    out["batched"] = quality
    return out


def mimo_grid_leg(args):
    """Detection quality over the MIMO grid (Fig. 5 / Table 1 sizes extended to
    Nt = 32, 64; workloads.mimo.grid_points()): Nt = Nr in {8, 16, 32, 64} x
    {4, 16}-QAM x Eb/N0 in {10, 15, 20, 25} dB, DI mapping, 32 trials, the
    steps of Table 1 doubled per doubling of Nt, beta = 1, xi = 2, gamma 0.05
    -> 0.3.  Per point: `channels` seeded channels in one batched launch per
    MFMA precision (FP8, BF16) and, on the first 64 of them, the plain FP32
    kernel; symbol and bit error rates against the transmitted symbols, the
    sliced MMSE estimate, and, from tests/golden/mimo_grid_ref.json (written
    by the CPU oracle): the binary64 oracle's own PIMI dynamics on those 64
    channels and exact ML detection where it is enumerable.  Energy gap: the
    mean over those 64 channels of (E of the GPU's best state - E of the
    oracle's best state) in the Eq. (1) units of the instance, and the share
    of channels where the GPU's is not higher."""
    import paper_2604_17109_amd as pim
    import workloads as w
    path = os.path.join(GOLDEN, "mimo_grid_ref.json")
    ref = {(r["nt"], r["qam"], r["ebn0_db"]): r for r in json.load(open(path))["points"]} \
        if os.path.exists(path) else {}
    ztab = w.gauss_table(8)
    C, R = args.grid_channels, 32
    rows = []
    t_start = time.perf_counter()
    for nt, qam, db, T in w.mimo.grid_points():
        beta, eta = w.constant(T, 1.0), w.mimo_eta(T, 0.05, 0.3)
        probs = [w.mimo.mimo_problem(nt, nt, qam, db, seed=w.mimo.GRID_SEED, index=k) for k in range(C)]
        maps = [pim.mimo_ising(p["H"], p["y"], qam, "di", p["esn0"]) for p in probs]
        sym = sum(p["nt"] for p in probs)
        bits = sym * w.mimo.bits_per_symbol(qam)

        def rates(dets, idx):
            se = be = 0
            for k, s_ in zip(idx, dets):
                x = pim.mimo_decode(maps[k][2], s_, qam, "di")
                se += int(np.count_nonzero(x != probs[k]["x"]))
                be += int(np.count_nonzero(w.mimo.bits_from_symbols(x, qam) != probs[k]["bits"]))
            ns_ = len(idx) * nt
            return se / ns_, be / (ns_ * w.mimo.bits_per_symbol(qam))

        row = {"nt": nt, "qam": qam, "ebn0_db": db, "steps": T, "channels": C, "n": maps[0][0].shape[0]}
        energies = {}
        for name, prec, kern, cnt in (("fp8", "fp8", "mfma", C), ("bf16", "bf16", "mfma", C),
                                      ("plain_f32", "fp8", "plain", min(C, 64))):
            insts = [pim.Instance(maps[k][0], maps[k][1], j_scale=1.0, xi=2.0, noise_table=ztab, rng_stream=k,
                                  prec=prec) for k in range(cnt)]
            b = pim.Batch(insts, R).run(beta, eta, seed=11, kernel=kern)
            best = [b.best(k) for k in range(cnt)]
            row[f"{name}_ser"], row[f"{name}_ber"] = rates([x[0] for x in best], range(cnt))
            if cnt > 64:  # the oracle's subset too, for a like-for-like comparison
                row[f"{name}_ser_first64"], row[f"{name}_ber_first64"] = rates([x[0] for x in best[:64]], range(64))
            row[f"{name}_kernel_ms"] = b.kernel_ms()
            energies[name] = np.array([x[1] for x in best[:64]])
            b.close()
            for i in insts:
                i.close()
        se = be = 0
        for k, p in enumerate(probs):
            x = maps[k][2][:nt] + 1j * maps[k][2][nt:]
            se += int(np.count_nonzero(x != p["x"]))
            be += int(np.count_nonzero(w.mimo.bits_from_symbols(x, qam) != p["bits"]))
        row["mmse_ser"], row["mmse_ber"] = se / sym, be / bits
        g = ref.get((nt, qam, db))
        if g and C >= g["channels"]:
            m = g["channels"]
            row["oracle_channels"] = m
            row["oracle_ser"], row["oracle_ber"] = g["oracle_ser"], g["oracle_ber"]
            row["ml_ser"], row["ml_ber"] = g["ml_ser"], g["ml_ber"]
            eo = np.array(g["oracle_best_energy"][:m])
            for name in ("fp8", "bf16", "plain_f32"):
                d = energies[name][:m] - eo
                row[f"{name}_energy_gap_mean"] = float(d.mean())
                row[f"{name}_not_above_oracle"] = float(np.mean(d <= 1e-9 * np.abs(eo)))
        rows.append(row)
    return {"workload": "MIMO detection grid, Nt = Nr in {8, 16, 32, 64} x {4, 16}-QAM x {10, 15, 20, 25} dB, "
                        f"DI mapping, {C} channels per point ({min(C, 64)} for the plain kernel), 32 trials",
            "reference": "tests/golden/mimo_grid_ref.json (binary64 oracle dynamics and ML on the first 64 "
                         "channels)" if ref else None,
            "seconds": time.perf_counter() - t_start, "points": rows}


def uneven_leg(args):
    """Batched SK-1 with uneven N: 128 instances, N_k = [100, 200, 400, 800,
    1000][k mod 5], J = +-1, h = 0, c = 1/sqrt(N_k), xi = 0.5, 1024 replicas
    each, beta linear 0.1 -> 3.0 with eta = sqrt(beta / 5).  All instances run
    in one batch: one part per N, launched together as one captured graph, on
    e2m1 (FP4) operands (J = +-1 is exact in e2m1, results identical to int8):
    couplings in LDS for N <= 256, and the parts above as one launch over a
    longest-first work list.  The same graph on int8 operands is timed beside
    it and must give identical results.  Also each N bucket alone on both
    operand types, for per-N rates and MFMA fractions (2 N^2 ops per
    replica-step, against the int8 and the FP4 peaks)."""
    import paper_2604_17109_amd as pim
    import workloads as w
    sizes = [100, 200, 400, 800, 1000]
    count, R, T = 128, 1024, args.uneven_steps
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    ns = [sizes[k % 5] for k in range(count)]
    insts = [pim.Instance(*w.sk1(ns[k], seed=9, index=k), j_scale=1 / math.sqrt(ns[k]), xi=0.5,
                          noise_table=w.gauss_table(8), rng_stream=k) for k in range(count)]
    batch = pim.Batch(insts, R)
    waves = batch.tune(steps=100).tolist()
    batch.run(beta, eta, seed=1)  # warm-up; also the best energies found
    gpu = [batch.best(k)[1] for k in range(count)]
    e_sa = sa_reference_uneven(ns, 9)
    ref = [min(a, b) for a, b in zip(gpu, e_sa)] if e_sa else gpu
    tgt = [math.floor(0.999 * r) for r in ref]
    batch.run(beta, eta, seed=2, target=tgt, kernel="mfma")
    k8 = batch.kernel_ms()
    res8 = [batch.trials_of(k, spins=False) for k in range(count)]
    batch.run(beta, eta, seed=2, target=tgt, kernel="f4")
    kms = batch.kernel_ms()
    res4 = [batch.trials_of(k, spins=False) for k in range(count)]
    same = all(np.array_equal(a[key], b[key]) for a, b in zip(res4, res8)
               for key in ("e_best", "t_best", "first_hit", "e_final"))
    updates = float(sum(ns)) * R * T
    ops = float(sum(2 * n * n for n in ns)) * R * (T + 1)
    hits = [(r["first_hit"] >= 0).mean() for r in res4]
    out = {"workload": f"{count} SK-1 instances, N in {sizes}, {R} replicas x {T} steps, one graph launch",
           "kernel": "e2m1 (FP4) MFMA: couplings in LDS for N <= 256, streamed above (one launch over all such parts)",
           "kernel_ms": kms, "spin_updates_per_s": updates / (kms / 1e3),
           "int8_mfma_frac": ops / (kms / 1e3) / INT8_MFMA_PEAK,
           "int8_operands": {"kernel_ms": k8, "spin_updates_per_s": updates / (k8 / 1e3),
                             "int8_mfma_frac": ops / (k8 / 1e3) / INT8_MFMA_PEAK},
           "identical_to_int8_operands": bool(same),
           "waves_per_workgroup": dict(zip(map(str, sizes), waves)),
           "p_bar_relaxed": float(np.mean(hits)),
           "criterion": ("E <= floor(0.999 * min(simulated-annealing reference, best of the warm-up run))" if e_sa
                         else "E <= floor(0.999 * best of the warm-up run)"), "per_n": {}}
    batch.close()
    for n in sizes:
        sub = [i for i, m in zip(insts, ns) if m == n]
        sub_tgt = [t for t, m in zip(tgt, ns) if m == n]
        b = pim.Batch(sub, R)
        b.run(beta, eta, seed=2, kernel="mfma")
        b.run(beta, eta, seed=2, target=sub_tgt, kernel="mfma")
        k8n = b.kernel_ms()
        b.run(beta, eta, seed=2, kernel="f4")
        b.run(beta, eta, seed=2, target=sub_tgt, kernel="f4")
        k = b.kernel_ms()
        u = float(len(sub)) * n * R * T
        o = 2.0 * n * n * len(sub) * R * (T + 1)
        # success against the same thresholds: p_bar, n99 and TTS99 with all
        # trials in flight, tau = this bucket's kernel time per trial-step
        p = float(np.mean([(b.trials_of(q, spins=False)["first_hit"] >= 0).mean() for q in range(len(sub))]))
        n99 = 1 if p >= 1 else (None if p <= 0 else math.ceil(math.log(0.01) / math.log(1 - p)))
        tau = (k / 1e3) / (len(sub) * R * T)
        out["per_n"][str(n)] = {"instances": len(sub), "kernel_ms": k, "spin_updates_per_s": u / (k / 1e3),
                                "int8_mfma_frac": o / (k / 1e3) / INT8_MFMA_PEAK, "p_bar_relaxed": p,
                                "n99": n99, "tts99_s": n99 * T * tau if n99 else None, "operands": "e2m1",
                                "fp4_mfma_frac": o / (k / 1e3) / FP4_MFMA_PEAK,
                                "int8_operands": {"kernel_ms": k8n, "spin_updates_per_s": u / (k8n / 1e3),
                                                  "int8_mfma_frac": o / (k8n / 1e3) / INT8_MFMA_PEAK}}
        if e_sa:
            out["per_n"][str(n)]["reference"] = reference_summary([g for g, m in zip(gpu, ns) if m == n],
                                                                  [a for a, m in zip(e_sa, ns) if m == n])
        b.close()
    for i in insts:
        i.close()
    return out


def serving_leg(args):
    """MIMO detection serving with continuous batching.  Two request mixes at
    Eb/N0 = 20 dB, DI mapping (N = 4 Nt spins), 32 trials x 64 steps each,
    FP8 MFMA sweep, binary64 re-rank, served by the request server:
    * "5g": Nt = Nr in {8, 16} x {4-QAM, 16-QAM} (N = 32, 64), the sizes the
      paper's real-time design targets;
    * "full": Nt = Nr in {8, 16, 32, 64} x {4-QAM, 16-QAM} (N = 32 ... 256).
    A request is the detection problem itself (H, y, modulation, Es/N0); the
    server stages H and y and builds the Ising instance (J, h, x_m) in binary64
    on the device.  Poisson arrivals at each rate (the paper's protocol: 10^5
    requests, Suppl. "Throughput measurement"); latency from arrival to a
    host-readable result (p50 / p99) with its split into stages, sustained
    throughput, and the share finished within the 1 ms slot budget of 5G NR
    at 15 kHz subcarrier spacing (Suppl. "Throughput requirement for LTE/5G
    systems").  A request's result does not depend on what else is in flight
    (its noise stream is its id): every rate must return the same states."""
    import paper_2604_17109_amd as pim
    import workloads as w
    cfg = MIMO
    T = cfg["steps"]
    beta = w.constant(T, cfg["beta"])
    eta = w.mimo_eta(T, *cfg["gamma"])
    M = args.serving_requests
    out = {}
    for mix, nts, rates in (("5g", (8, 16), (1e4, 1e5, 1e6)), ("full", (8, 16, 32, 64), (1e4, 1e5))):
        if args.serving_mix not in ("both", mix):
            continue
        pairs = [(nt, q) for nt in nts for q in (4, 16)]
        probs = []
        for k in range(M):
            nt, q = pairs[k % len(pairs)]
            probs.append(w.mimo.mimo_problem(nt, nt, q, 20.0, seed=23, index=k))
        Hc = [w.mimo.interleaved(p["H"]) for p in probs]
        yc = [w.mimo.interleaved(p["y"]) for p in probs]
        dims = np.array([(p["nr"], p["nt"], p["qam"], pim.MIMO_DI) for p in probs], np.int32)
        esn0 = np.array([p["esn0"] for p in probs], np.float64)
        hp = np.fromiter((a.ctypes.data for a in Hc), dtype=np.uintp, count=M)
        yp = np.fromiter((a.ctypes.data for a in yc), dtype=np.uintp, count=M)
        ids = np.arange(M, dtype=np.uint32)
        ns = np.array([4 * p["nt"] for p in probs])
        res = {"workload": f"{M} requests uniform over Nt = Nr in {list(nts)} x {{4,16}}-QAM, 20 dB, DI mapping "
                           f"built on the device, N = {ns.min()}..{ns.max()}, {cfg['trials']} trials x {T} steps, fp8",
               "rates": {}}
        # per launch: up to 256 requests for the small 5G sizes (fewer, larger
        # launches at high rates); 64 for the full mix, whose 64x64 requests
        # make a 256-slot chunk hold 200 MB of staging
        mb = args.serving_batch or (256 if mix == "5g" else 64)
        pre = args.serving_prealloc or 16
        srv = pim.Server(max_n=int(ns.max()), trials=cfg["trials"], beta=beta, eta=eta, xi=cfg["xi"],
                         noise_table=w.gauss_table(8), prec="fp8", slots_per_class=4096, max_batch=mb,
                         streams=args.serving_streams, seed=11, max_wait_us=150.0, prealloc_chunks=pre, mimo=True)
        res["server"] = {"max_batch": mb, "prealloc_chunks": pre, "streams": args.serving_streams,
                         "max_wait_us": 150.0, "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])}
        srv.submit_mimo_raw(ids[:len(pairs)], dims[:len(pairs)], esn0[:len(pairs)], hp[:len(pairs)],
                            yp[:len(pairs)])  # warm-up: every size class once
        left = len(pairs)
        while left:
            srv.flush()
            left -= len(srv.poll_mimo(states=False)[0])
        rng = np.random.default_rng(29)

        def stream(arrive, count):
            # Poisson arrivals of requests 0..count-1: submit as they arrive,
            # launch, collect.  Returns, per request, the completion time, the
            # stage times (relative to t0): admitted by submit, launched by
            # flush, seen finished by poll (library clock), the final state
            # and x_m
            done_t = np.full(count, np.nan)
            stages = np.full((count, 3), np.nan)
            st_all = np.zeros((count, pim.MAX_N_LDS), np.int8)
            xm_all = np.zeros((count, pim.MAX_N_LDS // 2))
            nxt = finished = 0
            slow = {"submit": 0, "flush": 0, "poll": 0}  # calls that took over 1 ms
            t0 = time.perf_counter()
            while finished < count:
                now = time.perf_counter() - t0
                if nxt < count and arrive[nxt] <= now:
                    k = int(np.searchsorted(arrive[:count], now, side="right"))
                    nxt += srv.submit_mimo_raw(ids[nxt:k], dims[nxt:k], esn0[nxt:k], hp[nxt:k], yp[nxt:k])
                    slow["submit"] += (time.perf_counter() - t0 - now) > 1e-3
                t1 = time.perf_counter()
                srv.flush()
                t2 = time.perf_counter()
                got, st, _, xm, tm = srv.poll_mimo()
                slow["flush"] += (t2 - t1) > 1e-3
                slow["poll"] += (time.perf_counter() - t2) > 1e-3
                if len(got):
                    done_t[got] = time.perf_counter() - t0
                    stages[got] = tm - t0
                    st_all[got] = st
                    xm_all[got] = xm
                    finished += len(got)
            stream.slow = slow
            return done_t, stages, st_all, xm_all

        def attribution(arrive, done_t, stages, late, ns_arr):
            # time per stage (microseconds): arrival -> admitted (host loop and
            # submit), admitted -> launched (batching wait), launched -> seen
            # finished (device work and readback, polling granularity), seen
            # -> returned to the caller
            parts = np.stack([stages[:, 0] - arrive, stages[:, 1] - stages[:, 0], stages[:, 2] - stages[:, 1],
                              done_t - stages[:, 2]], axis=1) * 1e6
            names = ["arrival_to_admitted", "admitted_to_launched", "launched_to_finished", "finished_to_returned"]
            out = {"p50_us": dict(zip(names, np.percentile(parts, 50, axis=0).round(1).tolist())),
                   "p99_us": dict(zip(names, np.percentile(parts, 99, axis=0).round(1).tolist()))}
            if late.any():
                lp = parts[late]
                out["late_requests"] = int(late.sum())
                out["late_mean_us"] = dict(zip(names, lp.mean(axis=0).round(1).tolist()))
                out["late_dominant_stage"] = dict(zip(names, np.bincount(np.argmax(lp, axis=1),
                                                                         minlength=4).tolist()))
            # per request size: launched -> finished percentiles and late count
            out["by_n"] = {str(m): {"requests": int((ns_arr == m).sum()), "late": int(late[ns_arr == m].sum()),
                                    "launched_to_finished_p50_us": round(float(np.percentile(parts[ns_arr == m, 2], 50)), 1),
                                    "launched_to_finished_p99_us": round(float(np.percentile(parts[ns_arr == m, 2], 99)), 1)}
                           for m in sorted(set(ns_arr.tolist()))}
            return out

        # steady state first: a short unmeasured stream at the highest rate
        # lets the server grow its slot chunks to what the load needs
        warm = min(M, 2000)
        stream(np.cumsum(rng.exponential(1.0 / max(rates), size=warm)), warm)
        first = None
        for lam in rates:
            # the steady state of this rate: an unmeasured stream at it first
            stream(np.cumsum(rng.exponential(1.0 / lam, size=warm)), warm)
            arrive = np.cumsum(rng.exponential(1.0 / lam, size=M))
            gc.collect()
            gc.disable()  # no collector pauses inside the measured stream
            try:
                done_t, stages, st_all, xm_all = stream(arrive, M)
            finally:
                gc.enable()
            lat = (done_t - arrive) * 1e6
            rec = {"offered_req_per_s": lam, "served_req_per_s": M / float(np.nanmax(done_t) - arrive[0]),
                   "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
                   "within_1ms": float(np.mean(lat <= 1000.0)),
                   "stages": attribution(arrive, done_t, stages, lat > 1000.0, ns),
                   "host_calls_over_1ms": dict(stream.slow)}
            if first is None:
                se = be = 0
                for k, p in enumerate(probs):
                    x = pim.mimo_decode(xm_all[k, :2 * p["nt"]], st_all[k, :ns[k]], p["qam"], "di")
                    se += int(np.count_nonzero(x != p["x"]))
                    be += int(np.count_nonzero(w.mimo.bits_from_symbols(x, p["qam"]) != p["bits"]))
                rec["ser"] = se / float(sum(p["nt"] for p in probs))
                rec["ber"] = be / float(sum(p["nt"] * w.mimo.bits_per_symbol(p["qam"]) for p in probs))
                first = st_all
            else:
                rec["same_states_as_first_rate"] = float(np.mean(np.all(st_all == first, axis=1)))
            res["rates"][f"{lam:.0e}"] = rec
        srv.close()
        out[mix] = res
    return out


def comparison_leg():
    """The paper's comparison on the GPU (Fig. 2 / Suppl. "Estimation of
    optimal clock cycles to solution", "Quantifying coupled oscillatory
    dynamics"): PIMI with fully parallel updates against the conventional PIM
    with sequential updates (Eq. (3): xi = 0, uniform noise, one spin per
    step), on SK-1 instances of N = 20 ... 200, and the neighbour-triggered
    flip rate of the parallel dynamics against xi.

    Protocol of Eqs. (5)-(6): each method runs 1024 trials per instance at
    every anneal length T of its own grid (beta linear 0.1 -> 3.0 over T;
    PIMI T steps with eta = sqrt(beta / 5), xi = 0.5; the sequential PIM
    T = sweeps x N single-spin steps with eta = 1); success = E <=
    floor(0.999 H_ref) with H_ref = min(simulated-annealing reference, best
    energy either method found in a warm-up at its longest T); TTS99(T) =
    n99(T) x (kernel time / trials), the GPU time per trial run with all
    trials in flight, minimised over T per method (the Eq. (6) optimum); the
    speedup is the ratio of the two optima."""
    import paper_2604_17109_amd as pim
    import workloads as w
    R, count = 1024, 4
    par_grid = (100, 300, 1000, 3000, 10000)   # update steps
    seq_grid = (10, 30, 100, 300, 1000)        # sweeps of N single-spin steps
    rows = []
    for n in (20, 50, 100, 200):
        insts = [pim.Instance(*w.sk1(n, seed=5, index=k), j_scale=1 / math.sqrt(n), xi=0.5,
                              noise_table=w.gauss_table(8), rng_stream=k) for k in range(count)]
        seqi = [pim.Instance(*w.sk1(n, seed=5, index=k), j_scale=1 / math.sqrt(n), xi=0.0,
                             noise_table=w.uniform_table(8), rng_stream=k) for k in range(count)]
        bp = pim.Batch(insts, R)
        bs = pim.Batch(seqi, R)

        def par_sched(T):
            b = w.linear_beta(T, 0.1, 3.0)
            return b, w.eta_sqrt_beta_over_5(b)

        def seq_sched(T):
            return w.linear_beta(T * n, 0.1, 3.0), w.constant(T * n, 1.0)

        bp.run(*par_sched(par_grid[-1]), seed=3)
        bs.run(*seq_sched(seq_grid[-1]), seed=3, kernel="seq")
        gpu = [min(bp.best(k)[1], bs.best(k)[1]) for k in range(count)]
        e_sa = sa_reference("compare", n, 5, count)
        href = [min(a, b) for a, b in zip(gpu, e_sa)] if e_sa else gpu
        tgt = [math.floor(0.999 * r) for r in href]

        def scan(batch, grid, sched, kernel, unit):
            out = []
            for T in grid:
                batch.run(*sched(T), seed=4, kernel=kernel, target=tgt)
                kms = batch.kernel_ms()
                p = float(np.mean([(batch.trials_of(k, spins=False)["first_hit"] >= 0).mean()
                                   for k in range(count)]))
                m = n99_of(p)
                out.append({unit: T, "p_bar": p, "n99": m, "kernel_ms": kms,
                            "tts99_ms": m * kms / (count * R) if m else None,
                            f"{unit}_to_solution": m * T if m else None})
            fin = [r for r in out if r["tts99_ms"] is not None]
            return out, (min(fin, key=lambda r: r["tts99_ms"]) if fin else None)

        pg, popt = scan(bp, par_grid, par_sched, "mfma", "steps")
        sg, sopt = scan(bs, seq_grid, seq_sched, "seq", "sweeps")
        rows.append({"n": n, "instances": count, "trials": R,
                     "reference": reference_summary(gpu, e_sa) if e_sa else "best found by either method",
                     "parallel": {"grid": pg, "optimum": popt},
                     "sequential": {"grid": sg, "optimum": sopt},
                     "tts99_speedup_at_optima": (sopt["tts99_ms"] / popt["tts99_ms"]) if (popt and sopt) else None})
        bp.close()
        bs.close()
    # neighbour-triggered flip rate vs xi, SK-1 N = 200
    n, T, R2 = 200, 1000, 256
    J, h = w.sk1(n, seed=5, index=0)
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)
    pnt = {}
    for xi in (0.0, 0.2, 0.5, 0.8):
        inst = pim.Instance(J, h, j_scale=1 / math.sqrt(n), xi=xi, noise_table=w.gauss_table(8), rng_stream=0)
        b = pim.Batch([inst], R2).run(beta, eta, seed=1, record=True)
        num, den = b.flip_counts(0)
        with np.errstate(invalid="ignore", divide="ignore"):
            p = np.where(den > 0, num / np.maximum(den, 1), np.nan)
        pnt[str(xi)] = {f"t={t}": (None if np.isnan(p[t]) else round(float(p[t]), 4)) for t in (10, 250, 500, 750, 999)}
        pnt[str(xi)]["mean_second_half"] = round(float(np.nanmean(p[T // 2:])), 4)
        b.close()
    return {"tts99_parallel_vs_sequential": rows,
            "flip_rate_vs_xi": {"workload": f"SK-1 N={n}, {R2} trials x {T} steps", "p_nt": pnt}}


def config1_leg():
    """SK-1 N = 20 (16 instances, seed 1, J = +-1, h = 0): plain FP32 fully
    parallel inertial dynamics, 64 trials, beta linear 0.1 -> 3.0 over T, eta
    = sqrt(beta / 5), xi = 0.5, c = 1/sqrt(20); ground truth by brute force over
    the 2^20 states (tests/golden/sk20_ground_all.json, written by the oracle).
    Success = a trial reaches the exact ground energy (at N = 20 the relaxed
    0.999 threshold is the same integer); p_bar, n99 and TTS99 in steps
    (n99 x T) and in GPU time, over a grid of T.  The int8 MFMA kernel runs the
    T = 1000 case too; its first hits must equal the plain kernel's."""
    import paper_2604_17109_amd as pim
    import workloads as w
    gold = {r["index"]: r["e_gs"] for r in json.load(open(os.path.join(GOLDEN, "sk20_ground_all.json")))}
    n, R, count = 20, 64, 16
    insts = [pim.Instance(*w.sk1(n, seed=1, index=k), j_scale=1 / math.sqrt(n), xi=0.5,
                          noise_table=w.gauss_table(8), rng_stream=k) for k in range(count)]
    b = pim.Batch(insts, R)
    tgt = [gold[k] for k in range(count)]
    rows = []
    for T in (50, 100, 200, 500, 1000):
        beta = w.linear_beta(T, 0.1, 3.0)
        eta = w.eta_sqrt_beta_over_5(beta)
        b.run(beta, eta, seed=1, kernel="plain", target=tgt)
        kms = b.kernel_ms()
        fh = [b.trials_of(k, spins=False)["first_hit"] for k in range(count)]
        p = float(np.mean([(f >= 0).mean() for f in fh]))
        m = n99_of(p)
        rows.append({"steps": T, "p_bar": p, "instances_solved": int(sum((f >= 0).any() for f in fh)),
                     "n99": m, "steps_to_solution": m * T if m else None, "kernel_ms_plain": kms,
                     "tts99_us_plain": m * kms * 1e3 / (count * R) if m else None})
        if T == 1000:
            b.run(beta, eta, seed=1, kernel="mfma", target=tgt)
            fm = [b.trials_of(k, spins=False)["first_hit"] for k in range(count)]
            rows[-1]["mfma_same_first_hits"] = bool(all(np.array_equal(a, c) for a, c in zip(fh, fm)))
            rows[-1]["kernel_ms_mfma"] = b.kernel_ms()
    b.close()
    fin = [r for r in rows if r["n99"]]
    return {"workload": "SK-1 N=20, 16 instances x 64 trials, beta linear 0.1 -> 3.0, plain FP32 kernel",
            "ground_truth": "brute force over 2^20 states", "grid": rows,
            "min_steps_to_solution": min(fin, key=lambda r: r["steps_to_solution"]) if fin else None}


def main():
    args = parse()
    if args.core_only:
        args.no_mimo = args.no_serving = args.no_uneven = args.no_compare = args.no_cpu_baseline = True
        args.no_mimo_grid = True
        args.no_tts_scan = True
        args.plain_instances = 0
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sweep shards by "
              "instance and trial with no exchange between GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2604_17109_amd as pim
    import workloads as w

    torch.cuda.set_device(0)
    n, R, T, I = args.n, args.trials, args.sweeps, args.instances
    xi, c = 0.5, 1.0 / math.sqrt(n)
    ztab = w.gauss_table(8)
    insts = [pim.Instance(*w.sk1(n, seed=1, index=k), j_scale=c, xi=xi, levels=4, noise_table=ztab,
                          rng_stream=k) for k in range(I)]
    batch = pim.Batch(insts, R)
    beta = w.linear_beta(T, 0.1, 3.0)
    eta = w.eta_sqrt_beta_over_5(beta)

    def step(seed, target=None):
        batch.run(beta, eta, seed=seed, kernel=args.kernel, target=target)
        return [batch.best(k)[1] for k in range(I)]

    # warmup: also the best energy found per instance, one half of the
    # reference energy; the other half is the stored annealing reference
    ref_gpu = None
    for wi in range(max(1, args.warmup)):
        e = step(seed=1000 + wi)
        ref_gpu = e if ref_gpu is None else [min(a, b) for a, b in zip(ref_gpu, e)]
    e_sa = sa_reference("sk200", n, 1, I)
    href = [min(a, b) for a, b in zip(ref_gpu, e_sa)] if e_sa else list(ref_gpu)
    target = [int(math.floor(0.999 * r)) for r in href]  # relaxed success threshold, H < 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for si in range(args.steps):
        step(seed=1, target=target)
        kms.append(batch.kernel_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1000.0 * dt / args.steps
    updates = float(I) * R * T * n
    value = updates / (dt / args.steps)
    kernel_ms = float(np.mean(kms))

    # success statistics of the last timed run -> TTS99
    res = [batch.trials_of(k, spins=False) for k in range(I)]
    hits = [r["first_hit"] for r in res]
    p_bar = float(np.mean([(fh >= 0).mean() for fh in hits]))
    # strict: the trial's best energy reaches the reference energy itself
    p_strict = float(np.mean([(r["e_best"] <= hr).mean() for r, hr in zip(res, href)]))
    timed_best = [float(r["e_best"].min()) for r in res]
    n99 = (1 if p_bar >= 1 else (math.inf if p_bar <= 0 else math.ceil(math.log(0.01) / math.log(1 - p_bar))))
    tau = (kernel_ms / 1000.0) / (I * R * T)  # seconds per trial-step on the full batch
    tts99 = n99 * T * tau if n99 != math.inf else None
    # best energies of the timed run, kept for the plain-kernel comparison
    # (the scan below reruns the batch)
    timed_ebest = [batch.trials_of(q, spins=False)["e_best"] for q in range(min(args.plain_instances, I))]
    # the same timed protocol on e2m1 (FP4) operands: J = +-1 and the spins are
    # exact e2m1 values, so every trial must give the int8 run's results
    e2m1 = None
    if args.kernel == "mfma" and not args.core_only:
        timed_res = [(r["e_best"], r["t_best"], r["first_hit"]) for r in res]
        batch.run(beta, eta, seed=1, kernel="f4", target=target)  # warm-up
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        k4 = []
        for si in range(args.steps):
            batch.run(beta, eta, seed=1, kernel="f4", target=target)
            [batch.best(k) for k in range(I)]
            k4.append(batch.kernel_ms())
        torch.cuda.synchronize()
        dt4 = time.perf_counter() - t4
        kms4 = float(np.mean(k4))
        res4 = [batch.trials_of(k, spins=False) for k in range(I)]
        same4 = all(np.array_equal(a[0], b["e_best"]) and np.array_equal(a[1], b["t_best"]) and
                    np.array_equal(a[2], b["first_hit"]) for a, b in zip(timed_res, res4))
        ops4 = 2.0 * n * n * float(I) * R * (T + 1)
        e2m1 = {"value": updates / (dt4 / args.steps), "unit": "spin-updates/s", "ms_per_step": 1000.0 * dt4 / args.steps,
                "kernel_ms": kms4, "identical_to_int8": bool(same4),
                "tts99_s": n99 * T * (kms4 / 1000.0) / (I * R * T) if n99 != math.inf else None,
                "int8_mfma_frac": ops4 / (kms4 / 1e3) / INT8_MFMA_PEAK,
                "fp4_mfma_frac": ops4 / (kms4 / 1e3) / FP4_MFMA_PEAK,
                "note": "couplings +-1 and spins +-2 are exact e2m1 values; binary32 sums of integer products "
                        "below 2^24 are exact, so trajectories equal the int8 kernel's"}

    # TTS99 over the anneal length: the same batch and success threshold, a
    # linear 0.1 -> 3.0 schedule over each T (after the timed region)
    def tts_row(Ts, p, kms):
        n = 1 if p >= 1 else (math.inf if p <= 0 else math.ceil(math.log(0.01) / math.log(1 - p)))
        t = (kms / 1000.0) / (I * R * Ts) if kms > 0 else 0.0
        return {"steps": Ts, "p_bar": p, "n99": n if n != math.inf else None,
                "tts99_s": n * Ts * t if n != math.inf else None}

    scan = []
    if args.kernel == "mfma" and not args.no_tts_scan:
        for Ts in sorted({t for t in (250, 500, 1000, 2000, 5000) if t < T}):
            bs = w.linear_beta(Ts, 0.1, 3.0)
            batch.run(bs, w.eta_sqrt_beta_over_5(bs), seed=1, kernel=args.kernel, target=target)
            hs = [batch.trials_of(k, spins=False)["first_hit"] for k in range(I)]
            scan.append(tts_row(Ts, float(np.mean([(fh >= 0).mean() for fh in hs])), batch.kernel_ms()))
    scan.append(tts_row(T, p_bar, kernel_ms))
    finite = [r for r in scan if r["tts99_s"] is not None]
    tts_best = min(finite, key=lambda r: r["tts99_s"]) if finite else None

    # roofline of the sweep kernel (algorithmic counts per launch)
    contractions = float(I) * R * (T + 1)
    mfma_ops = 2.0 * n * n * contractions
    # algorithmic 32-bit lane-ops per spin update: Philox4x32-10 share
    # (10 rounds x (2 widening multiplies + 2 three-way xors) / 16 values)
    # 2.5, threshold address + compare 2, spin pack 1, energy multiply-add 1
    alu_per_update = 6.5
    alu_ops = alu_per_update * updates
    kernel_s = kernel_ms / 1000.0
    # LDS traffic of the int8 kernel per wave (32 trials) and step: the J
    # fragments (Npad^2 bytes), 2-byte threshold lookups of the spins that carry
    # decisions, and the 1 KB table written for the next step
    nt = (n + 31) // 32
    rem = n - 32 * (nt - 1)
    tail = 16 if rem > 12 else 12 if rem > 8 else 8 if rem > 4 else 4
    lds_per_wave_step = nt * nt * 1024 + ((nt - 1) * 16 + tail) * 64 * 2 + 1024
    lds_bytes = lds_per_wave_step * float(I) * ((R + 31) // 32) * (T + 1)
    line = {
        "metric": "spin-updates/s (batched SK-1 N=200)",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4" if args.kernel == "f4" else "i8",
        "data": "synthetic",
        "config": {"workload": f"SK-1 N={n}, {I} instances x {R} trials x {T} steps, kernel {args.kernel}",
                   "instances": I, "trials": R, "steps_per_trial": T, "n": n, "parallelism": "single GPU"},
        "kernel_ms": kernel_ms,
        "tts99": {"p_bar": p_bar, "n99": n99 if n99 != math.inf else None, "tts99_s": tts99,
                  "criterion": ("E <= floor(0.999 * H_ref), H_ref = min(simulated-annealing reference of the "
                                "paper's SK-1 recipe, best of the warm-up runs)" if e_sa else
                                "E <= floor(0.999 * best energy of the warm-up runs) (no stored annealing "
                                "reference for this workload)"),
                  "steps": T, "p_bar_strict": p_strict,
                  "reference": (dict(reference_summary(ref_gpu, e_sa), timed_run=reference_summary(timed_best, e_sa),
                                     source="tests/golden/sa_ref.json: 10 Metropolis annealing runs per instance, "
                                            "T 5.0 -> 0.01 x0.995, 5*10^4 proposed flips per temperature")
                                if e_sa else None),
                  "over_steps": scan, "min_over_steps": tts_best},
        "roofline": {"bound": "alu", "achieved": alu_ops / kernel_s, "peak": VALU_PEAK, "unit": "lane-op/s",
                     "frac": alu_ops / kernel_s / VALU_PEAK,
                     "traffic": measured_traffic() if (args.n, args.trials, args.instances, args.sweeps)
                     == (200, 1024, 128, 10000) and args.kernel == "mfma" else None,
                     "algorithmic_per_update": alu_per_update},
        "roofline_mfma": {"bound": "mfma", "achieved": mfma_ops / kernel_s / 1e12, "peak": INT8_MFMA_PEAK / 1e12,
                          "unit": "TOP/s", "frac": mfma_ops / kernel_s / INT8_MFMA_PEAK},
        "roofline_fp4": ({"bound": "mfma", "achieved": mfma_ops / kernel_s / 1e12, "peak": FP4_MFMA_PEAK / 1e12,
                          "unit": "TOP/s", "frac": mfma_ops / kernel_s / FP4_MFMA_PEAK}
                         if args.kernel == "f4" else None),
        "lds": ({"achieved": lds_bytes / kernel_s / 1e9, "peak": LDS_PEAK / 1e9, "unit": "GB/s",
                 "frac": lds_bytes / kernel_s / LDS_PEAK, "bytes_per_wave_step": lds_per_wave_step}
                if args.kernel == "mfma" and n <= 256 else None),
    }
    if e2m1 is not None:
        e2m1["alu_frac"] = alu_ops / (e2m1["kernel_ms"] / 1e3) / VALU_PEAK
        line["e2m1"] = e2m1
    if args.plain_instances > 0 and args.kernel == "mfma":
        # the plain FP32 per-instance kernel on the first instances of the same
        # batch (identical trajectories, so equal TTS99): one launch per instance
        k = min(args.plain_instances, I)
        pb = pim.Batch(insts[:k], R)
        pb.run(beta, eta, seed=1, kernel="plain", target=target[:k])
        pms = pb.kernel_ms()
        theirs = [pb.trials_of(q, spins=False)["e_best"] for q in range(k)]
        same = all(np.array_equal(a, b) for a, b in zip(timed_ebest, theirs))
        plain_rate = float(k) * R * T * n / (pms / 1000.0)
        line["plain_f32"] = {"instances": k, "kernel_ms": pms, "spin_updates_per_s": plain_rate,
                             "identical_results": bool(same),
                             "speedup_at_equal_tts99": (updates / (kernel_ms / 1000.0)) / plain_rate}
        pb.close()
    if not args.no_mimo:
        line["mimo"] = mimo_leg(args)
    if not args.no_mimo_grid:
        line["mimo_grid"] = mimo_grid_leg(args)
    if not args.no_serving:
        line["serving"] = serving_leg(args)
    if not args.no_uneven:
        line["uneven_n"] = uneven_leg(args)
    if not args.no_compare:
        line["comparison"] = comparison_leg()
        line["config1"] = config1_leg()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_trials, args.cpu_steps, xi, c)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
