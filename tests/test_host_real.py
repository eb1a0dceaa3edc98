"""Host-side pins of the real-valued path (no GPU): the FP8 / BF16 quantisers
against exhaustive nearest-value search over each format's code table, the
binary32 field thresholds against the binary64 rule, and the library's MIMO
mapping against the oracle's."""
import numpy as np
import pytest

import paper_2604_17109_amd as pim
import workloads as w
from oracle import mimo, pimi

RNG = np.random.default_rng(1234)


def _fp8_table():
    """All finite non-negative OCP e4m3 values with their codes, from the
    format definition: bias 7, 3 mantissa bits, subnormals at exponent 0,
    code 0x7F is NaN."""
    vals, codes = [], []
    for c in range(0x7F):
        e, m = c >> 3, c & 7
        vals.append(m / 8.0 * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7))
        codes.append(c)
    return np.array(vals), np.array(codes)


def _bf16_table():
    codes = np.arange(0, 0x7F80, dtype=np.uint32)  # non-negative finite
    vals = (codes << 16).view(np.float32).astype(np.float64)
    return vals, codes


def _nearest_even(x, vals, codes):
    """Round |x| to the nearest table value, ties to the even code, keep sign."""
    a = np.abs(x)
    i = np.clip(np.searchsorted(vals, a), 1, len(vals) - 1)
    lo, hi = vals[i - 1], vals[i]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (codes[i] % 2 == 0))
    q = np.where(pick_hi, hi, lo)
    q = np.where(a >= vals[-1], vals[-1], q)  # saturate
    return np.sign(x) * q


@pytest.mark.parametrize("prec", ["fp8", "bf16"])
def test_quantize_is_nearest_even(prec):
    vals, codes = _fp8_table() if prec == "fp8" else _bf16_table()
    n = 64
    J = RNG.standard_normal((n, n)) * np.exp(RNG.uniform(-9, 3, (n, n)))
    # exact midpoints between neighbouring representable values (ties)
    k = RNG.integers(1, len(vals) - 1, size=200)
    J.flat[:200] = (vals[k] + vals[k + 1]) / 2 * np.where(RNG.random(200) < 0.5, -1, 1)
    J = np.triu(J, 1)
    J = J + J.T
    out, scale = pim.quantize(J, prec)
    if prec == "fp8":
        assert scale == np.float32(np.abs(J).max() / 448.0)
    else:
        assert scale == 2.0 ** np.floor(np.log2(np.abs(J).max()))
    want = scale * _nearest_even(J / scale, vals, codes)
    assert np.array_equal(out, want)
    assert np.array_equal(out, out.T) and np.all(np.diag(out) == 0)


def test_quantize_tie_rounding_examples():
    # e4m3 around 1: neighbours 1, 1.125; 1.0625 is a tie -> even code (1.0)
    J = np.zeros((2, 2))
    J[0, 1] = J[1, 0] = 448.0  # scale 1
    out, scale = pim.quantize(J, "fp8")
    assert scale == 1.0 and out[0, 1] == 448.0
    J = np.array([[0, 448.0, 1.0625, 1.1875], [448.0, 0, 3e-3, 500.0 * 0 + 17.0],
                  [1.0625, 3e-3, 0, 0], [1.1875, 17.0, 0, 0]])
    out, _ = pim.quantize(J, "fp8")
    assert out[0, 2] == 1.0          # tie between 1.0 (even) and 1.125
    assert out[0, 3] == 1.25         # tie between 1.125 and 1.25 (even)
    assert out[1, 2] == 2.0 ** -9 * 2   # 3e-3 -> nearest subnormal multiple of 2^-9
    assert out[1, 3] == 16.0         # tie between 16 (even) and 18


def _rule_decision(I, s, u, beta, c, xi, eta, ztab, L):
    """Eq. (4) in binary64 on a binary32 field value (the oracle's LUT and sign)."""
    g = beta * c
    act = pimi.tanh_lut(g * np.float64(I), L)
    return int(pimi.spin_decision(act, s, xi, eta, ztab[u]))


CASES = [
    # c, xi, L, beta, eta, noise
    (1.0, 2.0, 4, 1.0, 0.3, "gauss"),
    (1.0, 2.0, 4, 1.0, 1.2, "gauss"),
    (0.37, 0.5, 4, 2.3, 0.7, "gauss"),
    (1.0, 0.0, 4, 1.0, 0.5, "uniform"),
    (0.125, 0.7, 8, 3.0, 0.0, "gauss"),
    (1.0, 2.0, 2, 0.0, 0.9, "gauss"),
    (2.0, 1.0, 16, 0.61, 2.5, "uniform"),
]


@pytest.mark.parametrize("case", CASES)
def test_real_table_reproduces_binary64_rule(case):
    c, xi, L, beta, eta, noise = case
    ztab = w.gauss_table(8) if noise == "gauss" else w.uniform_table(8)
    tab = pim.compile_table_real(16, c, xi, beta, eta, levels=L, noise_table=ztab)
    finite = np.unique(tab[np.isfinite(tab)])
    probes = [np.float32(0.0), np.float32(-0.0), np.float32(1e-30), np.float32(-1e-30)]
    for th in finite:
        probes += [th, np.nextafter(th, np.float32(-np.inf)), np.nextafter(th, np.float32(np.inf))]
    probes += list(RNG.standard_normal(200).astype(np.float32) * 5)
    for I in probes:
        I = np.float32(I)
        for s in (1, -1):
            for u in range(256):
                idx = 256 + (u if s == 1 else ~u)
                th = tab[idx]
                d = np.float32(I - th) if np.isfinite(th) else (np.float32(-np.inf) if th > 0 else np.float32(np.inf))
                got = -1 if np.signbit(d) else 1   # the kernel's sign-bit decision
                assert got == _rule_decision(I, s, u, beta, c, xi, eta, ztab, L), (I, s, u, th)


@pytest.mark.parametrize("mapping,qam,nt", [("ml", 4, 4), ("ml", 16, 3), ("di", 4, 4), ("di", 16, 8), ("di", 16, 2)])
def test_mimo_mapping_matches_oracle(mapping, qam, nt):
    for idx in range(3):
        p = w.mimo.mimo_problem(nt, nt + 1, qam, 14.0, seed=8, index=idx)
        J, h, xm = pim.mimo_ising(p["H"], p["y"], qam, mapping, p["esn0"])
        d = mimo.detector_instance(p, mapping)
        assert J.shape == d["J"].shape
        scale = np.abs(d["J"]).max()
        assert np.allclose(J, d["J"], rtol=0, atol=1e-12 * scale)
        assert np.allclose(h, d["h"], rtol=0, atol=1e-12 * np.abs(d["h"]).max())
        assert np.array_equal(xm, d["xm"])
        for _ in range(5):
            s = RNG.choice(np.array([-1, 1], np.int8), size=J.shape[0])
            assert np.array_equal(pim.mimo_decode(xm, s, qam, mapping), mimo.decode(d["xm"], d["T"], s, qam))


def test_mimo_mapping_rejects_a_singular_mmse_system():
    """Two equal channel columns and a regulariser 1/(Es/N0) below rounding:
    the LDL^T factorization's second pivot is exactly 0, which the mapping
    rejects; with Es/N0 = 10 the same channel maps, and its sliced MMSE
    estimate equals the oracle's (Suppl. "Baseline: linear MMSE detector")."""
    H = np.ones((2, 2), complex)
    y = np.array([1.0 + 1.0j, 2.0 - 1.0j])
    with pytest.raises(pim.PimError, match="positive definite"):
        pim.mimo_ising(H, y, 16, "di", 1e300)
    J, h, xm = pim.mimo_ising(H, y, 16, "di", 10.0)
    p = {"H": H, "y": y, "qam": 16, "esn0": 10.0, "nt": 2, "nr": 2}
    assert np.array_equal(xm, mimo.detector_instance(p, "di")["xm"])


def test_real_instance_validation():
    J = np.zeros((4, 4))
    J[0, 1] = 1.0
    with pytest.raises(pim.PimError, match="symmetric"):
        pim.validate(J, j_scale=1.0, xi=2.0, prec="fp8")
    J[1, 0] = 1.0
    assert pim.validate(J, j_scale=1.0, xi=2.0, prec="bf16") is None
    J2 = J.copy()
    J2[2, 2] = 0.5
    with pytest.raises(pim.PimError, match="diagonal"):
        pim.validate(J2, j_scale=1.0, xi=2.0, prec="fp8")
    J3 = J.copy()
    J3[0, 1] = J3[1, 0] = np.inf
    with pytest.raises(pim.PimError, match="finite"):
        pim.validate(J3, j_scale=1.0, xi=2.0, prec="fp8")
    with pytest.raises(pim.PimError, match="h\\[1\\]"):
        pim.validate(J, np.array([0.0, np.nan, 0, 0]), j_scale=1.0, xi=2.0, prec="fp8")
    with pytest.raises(pim.PimError, match="precision"):
        pim.validate(J, j_scale=1.0, xi=2.0, prec=7)
