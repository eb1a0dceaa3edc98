"""Synthetic uplink MIMO detection problems (Suppl. "MIMO problem definition",
"Uplink MIMO instance generation").

One problem is (H, x, y) of the complex model y = H x + n:

* H [Nr, Nt]: i.i.d. Rayleigh fading, H = (H_R + j H_I) / sqrt(2) with H_R, H_I
  standard normal, so every entry is CN(0, 1);
* x [Nt]: symbols of a square M-QAM constellation drawn uniformly by drawing
  the b = log2(M) information bits of each symbol uniformly; the real and the
  imaginary part each take one of the sqrt(M) odd-integer levels
  -(sqrt(M) - 1), ..., -1, 1, ..., sqrt(M) - 1, Gray coded per component;
* n: AWGN whose complex variance is set from Eb/N0 through the empirical
  received power of the noiseless vector: sigma^2 = E_y / (b * Eb/N0), with
  E_y = mean_i |(H x)_i|^2, and n = sqrt(sigma^2 / 2) (w_R + j w_I).

Every problem is a deterministic function of (seed, index) through NumPy's
PCG64, so tests and benchmarks regenerate identical inputs on any machine.
The module also holds the Gray bit labelling (both directions), which is part
of the input's definition, not of any detector.
"""
import numpy as np


def _rng(seed, index):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(index), 0x4D494D4F])))


def pam_levels(qam):
    """Odd-integer amplitude levels of one real component of square M-QAM."""
    m = int(round(np.sqrt(qam)))
    if m * m != qam or m < 2 or (m & (m - 1)):
        raise ValueError("qam must be a square power of two (4, 16, 64, ...)")
    return np.arange(-(m - 1), m, 2, dtype=np.int64)


def bits_per_symbol(qam):
    return int(round(np.log2(qam)))


def _component_bits(qam):
    return bits_per_symbol(qam) // 2


def levels_from_bits(bits, qam):
    """Gray labelling of one real component: the level with index g (in
    increasing amplitude order) carries the bit pattern g ^ (g >> 1), most
    significant bit first.  bits: int array [..., k] -> odd-integer levels [...]."""
    k = _component_bits(qam)
    bits = np.asarray(bits, dtype=np.int64)
    gray = np.zeros(bits.shape[:-1], dtype=np.int64)
    for i in range(k):
        gray = (gray << 1) | bits[..., i]
    g = gray.copy()  # inverse Gray code: g = gray ^ (gray >> 1) ^ (gray >> 2) ...
    shift = gray >> 1
    while np.any(shift):
        g ^= shift
        shift >>= 1
    return pam_levels(qam)[g]


def bits_from_levels(levels, qam):
    """Inverse of levels_from_bits: odd-integer levels [...] -> bits [..., k]."""
    k = _component_bits(qam)
    lv = pam_levels(qam)
    levels = np.asarray(levels, dtype=np.int64)
    g = np.searchsorted(lv, levels)
    if np.any(g >= len(lv)) or np.any(lv[np.minimum(g, len(lv) - 1)] != levels):
        raise ValueError("value is not a constellation level")
    gray = g ^ (g >> 1)
    return np.stack([(gray >> (k - 1 - i)) & 1 for i in range(k)], axis=-1)


def symbols_from_bits(bits, qam):
    """Information bits [Nt, b] (first half: real component, second half:
    imaginary component) -> complex symbols [Nt]."""
    k = _component_bits(qam)
    bits = np.asarray(bits, dtype=np.int64)
    return levels_from_bits(bits[:, :k], qam) + 1j * levels_from_bits(bits[:, k:], qam)


def bits_from_symbols(x, qam):
    """Complex constellation symbols [Nt] -> information bits [Nt, b]."""
    x = np.asarray(x)
    re = np.rint(x.real).astype(np.int64)
    im = np.rint(x.imag).astype(np.int64)
    return np.concatenate([bits_from_levels(re, qam), bits_from_levels(im, qam)], axis=-1)


def mimo_problem(nt, nr, qam, ebn0_db, seed=1, index=0):
    """One detection problem.  Returns a dict with complex H [nr, nt], the
    transmitted bits [nt, b] and symbols x [nt], the received y [nr], the
    complex noise variance sigma2 and the linear Eb/N0 and Es/N0."""
    rng = _rng(seed, index)
    b = bits_per_symbol(qam)
    H = (rng.standard_normal((nr, nt)) + 1j * rng.standard_normal((nr, nt))) / np.sqrt(2.0)
    bits = rng.integers(0, 2, size=(nt, b))
    x = symbols_from_bits(bits, qam)
    y_rec = H @ x
    e_y = float(np.mean(np.abs(y_rec) ** 2))
    ebn0 = 10.0 ** (float(ebn0_db) / 10.0)
    sigma2 = e_y / (b * ebn0)
    n = np.sqrt(sigma2 / 2.0) * (rng.standard_normal(nr) + 1j * rng.standard_normal(nr))
    return {"H": H, "bits": bits, "x": x, "y": y_rec + n, "sigma2": sigma2,
            "ebn0": ebn0, "esn0": b * ebn0, "qam": int(qam), "nt": int(nt), "nr": int(nr)}


def interleaved(z):
    """Complex array -> float64 array with a trailing (re, im) axis, row-major:
    the layout the C library takes for complex inputs."""
    z = np.asarray(z, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1))


# The detection grid of the MIMO benchmark (Fig. 5 / Table 1 sizes and SNRs
# extended to Nt = 32, 64): Nt = Nr, modulation, Eb/N0 in dB and the number of
# update steps (Table 1's 16 / 32 for 8x8 and 32 / 64 for 16x16 with 4- / 16-QAM,
# doubled for every doubling of Nt).  32 trials, DI mapping (N = 4 Nt spins).
GRID_SIZES = (8, 16, 32, 64)
GRID_QAMS = (4, 16)
GRID_SNRS_DB = (10.0, 15.0, 20.0, 25.0)
GRID_SEED = 31


def grid_steps(nt, qam):
    return (16 if qam == 4 else 32) * (nt // 8)


def grid_points():
    return [(nt, qam, db, grid_steps(nt, qam)) for nt in GRID_SIZES for qam in GRID_QAMS for db in GRID_SNRS_DB]
