"""Pins of the oracle's Philox4x32-10 and of the B-bit value extraction."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, uniform_bits, seed_key, DOMAIN_NOISE

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_matches_rocrand_philox(rocrand_ref):
    """AMD's rocRAND implements the same published bijection; compare on
    counters that exercise every word of the key and counter."""
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 1 << 32, size=(400, 6), dtype=np.uint64)
    rows[:4] = 0
    rows[1, :] = 0xFFFFFFFF
    rows[2, 2] = 1
    rows[3, 5] = 7
    # rocRAND takes the low counter words as an element offset (4 values per
    # counter), so c1 must stay below 2^30 for the offset to fit 64 bits.
    rows[:, 3] &= 0x3FFFFFFF
    inp = "\n".join(" ".join(f"{int(v):x}" for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    k0, k1 = rows[:, 0], rows[:, 1]
    got = np.stack(philox4x32_10(rows[:, 2], rows[:, 3], rows[:, 4], rows[:, 5], k0, k1), axis=1)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


def test_seed_key_split():
    assert seed_key(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)
    assert seed_key(5) == (5, 0)


@pytest.mark.parametrize("bits", [8, 16])
def test_extraction_is_little_endian_byte_view(bits):
    """The Q = 128/B values of a block are the output words read as a
    little-endian sequence of B-bit fields (checked through a byte view, not
    through shifts)."""
    seed, stream, trial, step = 99, 3, 11, 5
    q = 128 // bits
    spins = np.arange(5 * q)
    u = uniform_bits(seed, DOMAIN_NOISE, stream, trial, step, spins, bits)
    k0, k1 = seed_key(seed)
    for blk in range(5):
        words = philox4x32_10(blk, step, trial, (DOMAIN_NOISE << 24) | stream, k0, k1)
        raw = np.array([int(w) for w in words], dtype="<u4").view("<u1" if bits == 8 else "<u2")
        np.testing.assert_array_equal(u[blk * q:(blk + 1) * q], raw.astype(np.int64))


def test_uniformity_chi_square():
    """256-bin chi-square of 8-bit values over (trial, step, spin) grids."""
    trial = np.arange(64)[:, None, None]
    step = np.arange(50)[None, :, None]
    spin = np.arange(64)[None, None, :]
    u = uniform_bits(1, DOMAIN_NOISE, 0, trial, step, spin, 8).ravel()
    counts = np.bincount(u, minlength=256)
    exp = u.size / 256.0
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 255 degrees of freedom: mean 255, sd ~22.6; accept within ~5 sd
    assert 140 < chi2 < 370
    # neighbouring values in the stream are uncorrelated
    x = u.astype(np.float64) - 127.5
    r = (x[1:] * x[:-1]).mean() / x.var()
    assert abs(r) < 0.01


def test_streams_differ_by_each_key_component():
    base = uniform_bits(1, 0, 0, 0, 0, np.arange(64), 8)
    for kw in [dict(seed=2), dict(domain=1), dict(stream=1), dict(trial=1), dict(step=1)]:
        args = dict(seed=1, domain=0, stream=0, trial=0, step=0)
        args.update(kw)
        other = uniform_bits(args["seed"], args["domain"], args["stream"], args["trial"],
                             args["step"], np.arange(64), 8)
        assert (other != base).mean() > 0.9
