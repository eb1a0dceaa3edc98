"""Quantile tables for the B-bit noise index u in [0, 2^B).

A uniform B-bit integer u selects the noise sample Z[u]:

* Gaussian N(0, 1) (Eq. 4): Z[u] = Phi^-1((u + 0.5) / 2^B), the standard normal
  quantile at the midpoint of the u-th of 2^B equal-probability cells;
* uniform U(-1, 1) (Eq. 3): Z[u] = (2u + 1 - 2^B) / 2^B, the midpoint of the
  u-th of 2^B equal cells of [-1, 1] (exact in binary64).

Both tables are non-decreasing in u.  They are inputs: the caller hands the same
table to the oracle and to the library.
"""
import numpy as np
from scipy.special import ndtri


def gauss_table(bits=8):
    u = np.arange(1 << bits, dtype=np.float64)
    return ndtri((u + 0.5) / float(1 << bits))


def uniform_table(bits=8):
    u = np.arange(1 << bits, dtype=np.float64)
    return (2.0 * u + 1.0 - float(1 << bits)) / float(1 << bits)
