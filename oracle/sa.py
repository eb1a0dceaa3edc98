"""Simulated-annealing reference energies (the paper's ground-truth recipe).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): used by ``tests/``, by
the scripts under ``tests/golden/`` that write stored reference energies, and
never by the product path.

Suppl. "SK-1 instance generation", "Ground-truth computation": single-spin-flip
Metropolis simulated annealing from a random configuration, temperature
geometric from 5.0 to 0.01 with cooling factor 0.995, a fixed number of
proposed flips per temperature that grows with N, ten independent runs, the
lowest energy met in any run recorded as the reference energy.

The loop itself is plain C (``oracle/sa.c``, built with gcc into
``oracle/libsa.so``); this module compiles it when the library is missing or
older than its source, and wraps it.

Readings where the recipe is silent (each also listed with the design notes):
* the annealed energy is Eq. (1) of the instance with J scaled by the
  preprocessing normalisation c (1/sqrt(N) for SK-1), so a temperature is in
  the units of the normalised couplings; energies are reported in the integer
  units of J (exact);
* a proposal picks its spin uniformly at random;
* sizes between the printed ones take the budget of the next printed size
  above (N < 70: 10 N; N <= 100: 10^4; N <= 150: 2*10^4; larger: 5*10^4).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sa.c")
LIB = os.path.join(HERE, "libsa.so")

T_INIT, T_FINAL, ALPHA, RUNS = 5.0, 0.01, 0.995, 10

_lib = None


def build(force=False):
    """Compiles oracle/sa.c into oracle/libsa.so with gcc (plain C, -O2)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i8p = ctypes.POINTER(ctypes.c_int8)
        lib.sa_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.sa_philox4x32_10.restype = None
        lib.sa_count_temperatures.argtypes = [ctypes.c_double] * 3
        lib.sa_count_temperatures.restype = ctypes.c_int64
        lib.sa_anneal.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                  i64p, i8p, i64p, i64p]
        lib.sa_anneal.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox(ctr, key):
    """The C generator's Philox4x32-10 on one counter (4 words) and key (2)."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().sa_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def count_temperatures(t_init=T_INIT, t_final=T_FINAL, alpha=ALPHA):
    return int(_load().sa_count_temperatures(t_init, t_final, alpha))


def flips_per_temperature(n):
    """Proposed flips per temperature for size N (see the module notes)."""
    n = int(n)
    if n < 70:
        return 10 * n
    if n <= 100:
        return 10_000
    if n <= 150:
        return 20_000
    return 50_000


def _instance(J, h):
    J = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    n = J.shape[0]
    h = np.zeros(n, np.int32) if h is None else np.ascontiguousarray(np.asarray(h, dtype=np.int32))
    if J.shape != (n, n) or h.shape != (n,):
        raise ValueError("J must be N x N and h length N")
    return J, h, n


def anneal(J, h, c, runs=RUNS, flips=None, seed=1, stream=0, t_init=T_INIT, t_final=T_FINAL, alpha=ALPHA,
           hist=None):
    """Runs the recipe; returns (lowest energy over all runs (int), one state
    with it (int8 [N]), per-run lowest energies (int64 [runs])).  ``hist``: an
    int64 array of 2^N visit counts to fill (N <= 20), or None."""
    J, h, n = _instance(J, h)
    if hist is not None:
        if hist.dtype != np.int64 or hist.shape != (1 << n,) or not hist.flags.c_contiguous:
            raise ValueError("hist must be a contiguous int64 array of 2^N counts")
        hist = _ptr(hist, ctypes.c_int64)
    flips = flips_per_temperature(n) if flips is None else int(flips)
    best = ctypes.c_int64(0)
    state = np.zeros(n, dtype=np.int8)
    per_run = np.zeros(runs, dtype=np.int64)
    rc = _load().sa_anneal(n, _ptr(J, ctypes.c_int32), _ptr(h, ctypes.c_int32), float(c), t_init, t_final, alpha,
                           flips, int(runs), int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream), ctypes.byref(best),
                           _ptr(state, ctypes.c_int8), _ptr(per_run, ctypes.c_int64), hist)
    if rc != 0:
        raise ValueError(f"sa_anneal rejected its arguments (code {rc})")
    return int(best.value), state, per_run


def metropolis_histogram(J, h, c, temp, proposals, seed=1, stream=0):
    """The anneal's own loop held at one temperature (T_init = T_final): visit
    counts of every configuration (index sum_i [s_i = +1] 2^i) after each of
    `proposals` Metropolis proposals, N <= 20."""
    J, h, n = _instance(J, h)
    hist = np.zeros(1 << n, dtype=np.int64)
    _, _, _ = anneal(J, h, c, runs=1, flips=proposals, seed=seed, stream=stream, t_init=temp, t_final=temp,
                     alpha=0.5, hist=hist)
    return hist
