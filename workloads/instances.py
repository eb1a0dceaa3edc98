"""Synthetic dense Ising instances.

* SK-1 (Suppl. "SK-1 instance generation"): symmetric J with every off-diagonal
  entry +1 or -1 with equal probability, zero diagonal, h = 0.
* Max-Cut (Suppl. "Max-Cut instance generation"; Fig. 2a): Erdos-Renyi G(N, p)
  with p = 0.5 and unit weights, mapped to Ising form by J = -A, h = 0.

Every instance is a deterministic function of (seed, index) through NumPy's
PCG64 seeded with the pair, so the tests and the benchmark regenerate identical
inputs on any machine.
"""
import numpy as np


def _rng(seed, index):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(index)])))


def _symmetric_from_upper(upper_values, n, dtype=np.int8):
    j = np.zeros((n, n), dtype=dtype)
    iu = np.triu_indices(n, k=1)
    j[iu] = upper_values
    j[(iu[1], iu[0])] = upper_values
    return j


def sk1(n, seed=1, index=0):
    """SK-1 instance of size n: returns (J int8 [n, n], h int32 [n])."""
    rng = _rng(seed, index)
    m = n * (n - 1) // 2
    vals = np.where(rng.integers(0, 2, size=m) == 1, 1, -1).astype(np.int8)
    return _symmetric_from_upper(vals, n), np.zeros(n, dtype=np.int32)


def maxcut(n, seed=1, index=0, p=0.5):
    """Unweighted G(n, p) Max-Cut instance mapped to J = -A, h = 0."""
    rng = _rng(seed, index)
    m = n * (n - 1) // 2
    edges = (rng.random(m) < p).astype(np.int8)
    return _symmetric_from_upper(-edges, n), np.zeros(n, dtype=np.int32)


def random_int8(n, seed=1, index=0, jmax=127, hmax=0, density=1.0):
    """General integer instance: symmetric J with entries uniform in
    [-jmax, jmax] (zero with probability 1 - density), zero diagonal, and h
    uniform in [-hmax, hmax]."""
    rng = _rng(seed, index)
    m = n * (n - 1) // 2
    vals = rng.integers(-jmax, jmax + 1, size=m)
    if density < 1.0:
        vals = np.where(rng.random(m) < density, vals, 0)
    j = _symmetric_from_upper(vals.astype(np.int8), n)
    h = rng.integers(-hmax, hmax + 1, size=n).astype(np.int32) if hmax > 0 else np.zeros(n, np.int32)
    return j, h


def dense_problem(kind, n, seed=1, index=0):
    if kind == "sk":
        return sk1(n, seed, index)
    if kind == "maxcut":
        return maxcut(n, seed, index)
    raise ValueError(f"unknown problem kind {kind!r}")
