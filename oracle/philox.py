"""Philox4x32-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel Random
Numbers: As Easy as 1, 2, 3", SC'11 -- the Philox-4x32 bijection with R = 10
rounds.  One round maps the counter (c0, c1, c2, c3) under the round key
(k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with multipliers M0 = 0xD2511F53 and M1 = 0xCD9E8D57; between rounds the key is
bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.  The output is
the counter after the tenth round.

The paper itself streams pre-generated Gaussian samples from on-board memory
(Suppl. "PIMI FPGA implementation for Max-cut and SK-1", "Matrix, state, and
schedule storage"); a counter-based generator keyed on (seed, trial, step,
spin) replaces that table so every sample is reproducible without storing it.

Everything here is plain NumPy on uint64 arrays holding 32-bit values.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
ROUNDS = 10


def _mulhilo(m, x):
    """32x32 -> 64-bit product split into (hi, lo) 32-bit halves."""
    p = m * x  # both < 2^32, so the product fits in uint64 exactly
    return p >> np.uint64(32), p & MASK32


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply the ten-round Philox-4x32 bijection.

    Counter words c0..c3 may be NumPy arrays (broadcast together); the key
    words k0, k1 are Python ints or arrays.  Returns four uint64 arrays that
    hold the 32-bit output words x0..x3.
    """
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for r in range(ROUNDS):
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r + 1 < ROUNDS:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
    return c0, c1, c2, c3


# Counter domains: the fourth counter word carries (domain << 24) | stream id.
DOMAIN_NOISE = 0
DOMAIN_INIT = 1


def seed_key(seed):
    """64-bit seed -> Philox key words (low half, high half)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform_bits(seed, domain, stream, trial, step, spin, bits):
    """B-bit uniform integer for each (trial, step, spin), B in {8, 16}.

    Spin i of a trial draws from Philox block i // Q with Q = 128 / B values per
    block: the block index is counter word 0, the step counter word 1, the trial
    counter word 2 and (domain << 24) | stream counter word 3.  Within the block,
    value q = i % Q is field q % (32 / B) of output word q // (32 / B), fields
    counted from the least significant bits.
    """
    if bits not in (8, 16):
        raise ValueError("bits must be 8 or 16")
    if not 0 <= int(stream) < (1 << 24):
        raise ValueError("stream id must fit in 24 bits")
    q_per_block = 128 // bits
    per_word = 32 // bits
    trial = np.asarray(trial, dtype=np.uint64)
    step = np.asarray(step, dtype=np.uint64)
    spin = np.asarray(spin, dtype=np.int64)
    trial, step, spin = np.broadcast_arrays(trial, step, spin)
    block = (spin // q_per_block).astype(np.uint64)
    q = spin % q_per_block
    k0, k1 = seed_key(seed)
    c3 = np.uint64((int(domain) << 24) | int(stream))
    x = philox4x32_10(block, step, trial, c3, k0, k1)
    words = np.stack(x, axis=0)  # (4, ...)
    w = (q // per_word).astype(np.int64)
    f = (q % per_word).astype(np.uint64)
    word = np.take_along_axis(words, w[None, ...], axis=0)[0]
    return ((word >> (np.uint64(bits) * f)) & np.uint64((1 << bits) - 1)).astype(np.int64)
