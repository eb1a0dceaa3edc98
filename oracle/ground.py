"""Exact ground states by enumeration, for small instances.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The minimum of Eq. (1) over all 2^N configurations, by brute force: the
configurations are enumerated in chunks and their energies evaluated with the
field form -1/2 s^T J s - h^T s.  Feasible up to N ~ 22 on a laptop.
"""
import numpy as np


def _configs(n, start, stop):
    idx = np.arange(start, stop, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return (2 * bits - 1).astype(np.float64)  # [chunk, n], bit i -> spin i


def brute_force(J, h, chunk=1 << 16):
    """Returns (E_min, one minimising configuration as int64 [N], count of
    minimisers)."""
    J = np.asarray(J, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    n = J.shape[0]
    if n > 26:
        raise ValueError("brute force is limited to N <= 26")
    best = np.inf
    best_s = None
    count = 0
    total = 1 << n
    for start in range(0, total, chunk):
        S = _configs(n, start, min(total, start + chunk))
        e = -0.5 * np.einsum("ri,ij,rj->r", S, J, S) - S @ h
        e = np.rint(e)
        m = e.min()
        if m < best:
            best = m
            best_s = S[np.argmin(e)].astype(np.int64)
            count = int((e == m).sum())
        elif m == best:
            count += int((e == m).sum())
    return int(best), best_s, count
