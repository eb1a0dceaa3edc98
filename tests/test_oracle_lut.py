"""Pins of the L-level tanh lookup table (Algorithm "LUT-based tanh approximation")."""
import numpy as np
import pytest

from oracle import pimi


def test_four_level_table_values():
    # L = 4: breakpoints -1, -1/2, 0, 1/2, 1; levels -1, -1/3, 1/3, 1
    xs = [-5.0, -1.0000001, -1.0, -0.75, -0.5000001, -0.5, -0.1, 0.0, 0.25, 0.4999, 0.5, 0.9, 1.0, 1.0001, 7.0]
    want = [-1, -1, -1, -1, -1, -1 / 3, -1 / 3, 1 / 3, 1 / 3, 1 / 3, 1, 1, 1, 1, 1]
    np.testing.assert_allclose(pimi.tanh_lut(np.array(xs), 4), want, rtol=0, atol=1e-15)


def test_two_levels_is_a_sign_with_zero_up():
    x = np.array([-3, -1e-12, 0.0, 1e-12, 2])
    np.testing.assert_array_equal(pimi.tanh_lut(x, 2), [-1, -1, 1, 1, 1])


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 16])
def test_levels_uniform_and_saturating(L):
    lev = pimi.lut_levels(L)
    assert lev[0] == -1.0 and lev[-1] == 1.0
    np.testing.assert_allclose(np.diff(lev), 2.0 / (L - 1))
    b = pimi.lut_breakpoints(L)
    assert b[0] == -1.0 and b[-1] == 1.0 and len(b) == L + 1
    np.testing.assert_allclose(np.diff(b), 2.0 / L)
    x = np.linspace(-3, 3, 20001)
    y = pimi.tanh_lut(x, L)
    assert np.all(np.diff(y) >= 0)  # monotone
    assert set(np.round(np.unique(y), 12)) <= set(np.round(lev, 12))
    # each level is taken on exactly one bin of width 2/L inside [-1, 1]
    for k in range(L):
        mid = -1.0 + (2 * k + 1) / L
        assert pimi.tanh_lut(np.array([mid]), L)[0] == pytest.approx(lev[k])


def test_approximates_tanh_within_bin_width():
    # the paper uses the table in place of tanh: with many levels the two agree
    # on [-1, 1] to about one bin width (the table is a quantised identity there)
    x = np.linspace(-1, 1, 1001)
    err = np.abs(pimi.tanh_lut(x, 64) - x).max()
    assert err <= 2.0 / 63 + 1e-12
