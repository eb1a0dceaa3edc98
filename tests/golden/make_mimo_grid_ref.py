"""Writes tests/golden/mimo_grid_ref.json: reference detection quality on the
MIMO benchmark grid, from the oracle only.

For every grid point (workloads.mimo.grid_points(): Nt = Nr in {8, 16, 32, 64},
4- and 16-QAM, Eb/N0 10 / 15 / 20 / 25 dB) and the first CHANNELS channels
(workloads.mimo.mimo_problem(nt, nt, qam, db, seed=GRID_SEED, index=k)):

* the binary64 oracle's PIMI dynamics (Suppl. "PIMI FPGA implementation for
  MIMO detection": beta = 1, xi = 2, eta = sqrt(1 / (5 gamma)), gamma linear
  0.05 -> 0.3; 32 trials; DI mapping; Philox seed 11, noise stream = channel
  index): symbol and bit errors, and each channel's lowest Eq. (1) energy;
* exact ML detection by enumeration where it is small enough (4-QAM,
  Nt = 8: 4^8 symbol vectors): symbol and bit errors;
* the sliced MMSE estimate (Suppl. "Baseline: linear MMSE detector").

Run from the repository root (a few minutes on 8 cores):
    python tests/golden/make_mimo_grid_ref.py
"""
import json
import multiprocessing
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as w  # noqa: E402
from oracle import mimo, pimi  # noqa: E402

OUT = os.path.join(HERE, "mimo_grid_ref.json")
CHANNELS = 64
TRIALS = 32
SEED = 11


def one(point):
    nt, qam, db, steps = point
    beta, eta = w.constant(steps, 1.0), w.mimo_eta(steps, 0.05, 0.3)
    ztab = w.gauss_table(8)
    se = be = se_ml = be_ml = se_mmse = be_mmse = 0
    energies = []
    enumerable = qam == 4 and nt <= 8
    for k in range(CHANNELS):
        p = w.mimo.mimo_problem(nt, nt, qam, db, seed=w.mimo.GRID_SEED, index=k)
        d = mimo.detector_instance(p, "di")
        prob = pimi.RealProblem(d["J"], d["h"], 1.0, 2.0, 4, ztab)
        ref = pimi.run_parallel(prob, beta, eta, SEED, k, np.arange(TRIALS))
        e = pimi.energy_f64(d["J"], d["h"], ref["best_state"].astype(np.float64))
        a = int(np.argmin(e))
        energies.append(float(e[a]))
        x = mimo.decode(d["xm"], d["T"], ref["best_state"][:, a], qam)
        se += mimo.symbol_errors(p["x"], x)
        be += mimo.bit_errors(p["bits"], w.mimo.bits_from_symbols(x, qam))
        xm = mimo.complex_vector(d["xm"])
        se_mmse += mimo.symbol_errors(p["x"], xm)
        be_mmse += mimo.bit_errors(p["bits"], w.mimo.bits_from_symbols(xm, qam))
        if enumerable:
            x_ml, _ = mimo.ml_enumerate(p["H"], p["y"], qam)
            se_ml += mimo.symbol_errors(p["x"], x_ml)
            be_ml += mimo.bit_errors(p["bits"], w.mimo.bits_from_symbols(x_ml, qam))
    sym, bits = CHANNELS * nt, CHANNELS * nt * w.mimo.bits_per_symbol(qam)
    return {"nt": nt, "qam": qam, "ebn0_db": db, "steps": steps, "channels": CHANNELS,
            "oracle_ser": se / sym, "oracle_ber": be / bits, "mmse_ser": se_mmse / sym, "mmse_ber": be_mmse / bits,
            "ml_ser": se_ml / sym if enumerable else None, "ml_ber": be_ml / bits if enumerable else None,
            "oracle_best_energy": [float(f"{v:.15g}") for v in energies]}


def main():
    pts = w.mimo.grid_points()
    pts.sort(key=lambda p: -p[0] * p[3])  # largest first
    with multiprocessing.Pool(int(os.environ.get("WORKERS", "8"))) as pool:
        rows = []
        for r in pool.imap_unordered(one, pts):
            rows.append(r)
            print(f"[{len(rows)}/{len(pts)}] Nt={r['nt']} {r['qam']}-QAM {r['ebn0_db']} dB: oracle SER "
                  f"{r['oracle_ser']:.4f} MMSE {r['mmse_ser']:.4f} ML {r['ml_ser']}", flush=True)
    rows.sort(key=lambda r: (r["nt"], r["qam"], r["ebn0_db"]))
    data = {"recipe": {"source": "oracle/pimi.py RealProblem + oracle/mimo.py, DI mapping", "trials": TRIALS,
                       "seed": SEED, "channels_per_point": CHANNELS, "channel_seed": w.mimo.GRID_SEED,
                       "schedule": "beta = 1, xi = 2, eta = sqrt(1 / (5 gamma)), gamma linear 0.05 -> 0.3",
                       "writer": "tests/golden/make_mimo_grid_ref.py (oracle only)"},
            "points": rows}
    with open(OUT, "w") as f:
        json.dump(data, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
