"""Host-side tests of libpim.so that need no GPU: exported symbols, argument
validation, and the schedule compiler against the oracle's direct
binary64 evaluation of Eq. (4)."""
import os
import re

import numpy as np
import pytest

import workloads as w
from oracle import pimi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pim():
    import paper_2604_17109_amd as pim
    return pim


def test_library_exports_every_declared_symbol(pim):
    header = open(os.path.join(ROOT, "include", "pim.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(pim_[a-z_]+)\s*\(", header))
    declared -= {"pim_alloc_fn", "pim_free_fn"}
    assert declared == set(pim.EXPORTED)
    for name in declared:
        assert hasattr(pim.lib, name)
    assert pim.lib.pim_abi_version() == pim.ABI_VERSION == 2


def _compiled_decision(theta, umin, I, s, u):
    """s(t+1) = +1 iff u >= umin[2k + (s<0)] with k = #{j : I >= theta_j}: the
    contract of pim_compile_step's outputs."""
    k = (I[..., None] >= theta).sum(-1)
    return np.where(u >= umin[2 * k + (s < 0)], 1, -1)


CASES = [
    # (n, c, xi, L, noise, beta, eta)
    (20, 1 / np.sqrt(20), 0.5, 4, "gauss", 0.1, np.sqrt(0.1 / 5)),
    (200, 1 / np.sqrt(200), 0.5, 4, "gauss", 3.0, np.sqrt(3.0 / 5)),
    (200, 2 / np.sqrt(200), 0.7, 4, "gauss", 1.37, 0.52),
    (64, 0.25, 0.0, 4, "uniform", 0.2, 1.0),
    (64, 0.25, 1.0 / 3.0, 4, "gauss", 1.0, 0.0),      # exact ties (eta = 0)
    (50, 0.3, 0.2, 2, "gauss", 0.7, 0.9),
    (50, 0.3, 0.2, 3, "uniform", 0.7, 0.9),
    (50, 0.1, 0.45, 7, "gauss", 2.5, 0.3),
    (33, 0.5, 0.0, 4, "gauss", 0.0, 0.5),              # beta = 0
    (33, 0.5, 3.0, 4, "gauss", 1.0, 0.2),              # frozen by inertia
    (100, 1e-3, 0.5, 16, "gauss", 1.0, 0.7),           # thresholds beyond the field range
]


@pytest.mark.parametrize("case", CASES)
def test_compiled_thresholds_reproduce_direct_rule(pim, case):
    n, c, xi, L, noise, beta, eta = case
    ztab = w.gauss_table(8) if noise == "gauss" else w.uniform_table(8)
    theta, umin = pim.compile_step(n, c, xi, beta, eta, levels=L, noise_table=ztab)
    I = np.arange(-600, 601)[:, None, None]
    s = np.array([-1, 1])[None, :, None]
    u = np.arange(256)[None, None, :]
    I, s, u = np.broadcast_arrays(I, s, u)
    got = _compiled_decision(theta, umin, I, s, u)
    act = pimi.tanh_lut((beta * c) * I.astype(np.float64), L)
    want = pimi.spin_decision(act, s, xi, eta, ztab[u])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("case", CASES)
def test_kernel_table_reproduces_direct_rule(pim, case):
    """The 512-entry table the MFMA kernel reads: s(t+1) = +1 iff
    I >= table[256 + (u ^ s)], against the oracle's direct binary64 rule."""
    n, c, xi, L, noise, beta, eta = case
    ztab = w.gauss_table(8) if noise == "gauss" else w.uniform_table(8)
    tab = pim.compile_table(n, c, xi, beta, eta, levels=L, noise_table=ztab).astype(np.int64)
    I = np.arange(-600, 601)[:, None, None]
    s = np.array([-1, 1])[None, :, None]
    u = np.arange(256)[None, None, :]
    I, s, u = np.broadcast_arrays(I, s, u)
    got = np.where(I >= tab[256 + (u ^ s)], 1, -1)
    act = pimi.tanh_lut((beta * c) * I.astype(np.float64), L)
    want = pimi.spin_decision(act, s, xi, eta, ztab[u])
    assert np.array_equal(got, want)


def test_threshold_clamp_range(pim):
    # tiny g: thresholds lie far outside any admissible field and clamp
    theta, _ = pim.compile_step(10, 1e-9, 0.5, 1.0, 0.5, levels=4, noise_table=w.gauss_table(8))
    assert theta[0] == -32768 and theta[2] == 32767
    theta, umin = pim.compile_step(10, 0.5, 0.5, 0.0, 0.5, levels=4, noise_table=w.gauss_table(8))
    # beta = 0: x = 0 for all I -> bins with b_j <= 0 always counted
    np.testing.assert_array_equal(theta, [-32768, -32768, 32767])


def test_builtin_noise_tables_match_reference_tables(pim):
    """The library's own tables (used when the caller passes none) agree with
    scipy's normal quantile to a few ulp and exactly for the uniform law, and
    compile to identical thresholds on the configured schedules."""
    ztab = w.gauss_table(8)
    for (n, c, xi, L, noise, beta, eta) in CASES:
        ref = ztab if noise == "gauss" else w.uniform_table(8)
        t1, u1 = pim.compile_step(n, c, xi, beta, eta, levels=L, noise=noise)
        t2, u2 = pim.compile_step(n, c, xi, beta, eta, levels=L, noise_table=ref)
        np.testing.assert_array_equal(t1, t2)
        np.testing.assert_array_equal(u1, u2)
    # schedule sweep of the benchmark workload
    beta = w.linear_beta(2000)
    eta = w.eta_sqrt_beta_over_5(beta)
    for b, e in zip(beta[::7], eta[::7]):
        a = pim.compile_step(200, 1 / np.sqrt(200), 0.5, b, e, noise="gauss")
        r = pim.compile_step(200, 1 / np.sqrt(200), 0.5, b, e, noise_table=ztab)
        np.testing.assert_array_equal(a[1], r[1])


@pytest.mark.parametrize("bad,status,frag", [
    ("asym", 1, "symmetric"), ("diag", 1, "diagonal"), ("m128", 1, "-128"),
    ("rowbound", 1, "exceeds"), ("n0", 1, "n = 0"), ("L1", 1, "levels"),
    ("bits16", 2, "noise_bits"), ("nanxi", 1, "xi"), ("negc", 1, "j_scale"),
    ("nonmono", 1, "non-decreasing"), ("stream", 1, "rng_stream"),
])
def test_create_rejects_invalid_arguments(pim, bad, status, frag):
    n = 8
    J = w.sk1(n, seed=1)[0]
    h = None
    kw = dict(j_scale=0.5, xi=0.5, levels=4)
    if bad == "asym":
        J = J.copy(); J[0, 1] = -J[0, 1]
    elif bad == "diag":
        J = J.copy(); J[2, 2] = 1
    elif bad == "m128":
        J = J.copy(); J[0, 1] = J[1, 0] = -128
    elif bad == "rowbound":
        J = np.full((n, n), 100, np.int8) - np.diag(np.full(n, 100, np.int8))
        h = np.full(n, 32766, np.int32)
    elif bad == "n0":
        J = np.zeros((0, 0), np.int8)
    elif bad == "L1":
        kw["levels"] = 1
    elif bad == "bits16":
        kw["noise_bits"] = 16
    elif bad == "nanxi":
        kw["xi"] = float("nan")
    elif bad == "negc":
        kw["j_scale"] = -1.0
    elif bad == "nonmono":
        kw["noise_table"] = w.gauss_table(8)[::-1].copy()
    elif bad == "stream":
        pass
    if bad == "stream":
        p, keep = pim.make_params(n, 0.5, 0.5, rng_stream=1 << 24)
        import ctypes
        handle = ctypes.c_void_p()
        st = pim.lib.pim_create(J.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), None, ctypes.byref(p),
                                None, ctypes.byref(handle))
        assert st == status and frag in pim.lib.pim_last_error().decode()
        return
    with pytest.raises(pim.PimError) as ei:
        pim.validate(J, h, **kw)
    assert ei.value.status == status
    assert frag in str(ei.value)


def test_valid_arguments_pass_validation(pim):
    J, h = w.random_int8(40, seed=2, jmax=127, hmax=100)
    # row bound sum |J| + |h| stays below the field limit for n = 40
    assert pim.validate(J, h, j_scale=0.1, xi=0.3, levels=5) is None
    assert pim.validate(w.sk1(256)[0], j_scale=1 / 16, xi=0.5) is None


def _server_config(pim, keep, **over):
    import ctypes
    T = over.pop("steps", 16)
    beta = np.ascontiguousarray(over.pop("beta", np.full(T, 1.0)), dtype=np.float64)
    eta = np.ascontiguousarray(over.pop("eta", np.full(T, 0.3)), dtype=np.float64)
    keep += [beta, eta]
    c = pim.ServerConfig()
    c.max_n, c.slots_per_class, c.max_batch, c.trials, c.steps = 64, 64, 16, 32, T
    c.beta = beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.eta = eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.j_scale, c.xi, c.levels, c.noise, c.prec, c.streams = 1.0, 2.0, 4, 0, pim.PREC_FP8, 2
    for k, v in over.items():
        if k == "null_beta":
            c.beta = None
        else:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("over,frag", [
    ({"max_n": 0}, "max_n"), ({"max_n": 257}, "max_n"), ({"trials": 0}, "trials and steps"),
    ({"steps": 0}, "trials and steps"), ({"null_beta": 1}, "beta and eta"), ({"prec": 7}, "precision"),
    ({"streams": 0}, "streams"), ({"streams": 17}, "streams"), ({"max_batch": 0}, "max_batch"),
    ({"max_batch": 65536, "slots_per_class": 70000}, "max_batch"), ({"slots_per_class": 8}, "slots_per_class"),
    ({"beta": np.r_[np.ones(15), -1.0]}, "beta[15]"), ({"eta": np.r_[np.nan, np.ones(15)]}, "beta[0]"),
    ({"levels": 1}, "levels"),
])
def test_server_create_rejects_invalid_config(pim, over, frag):
    """Configuration errors are reported before any device work (no GPU here),
    and the handle stays NULL."""
    import ctypes
    keep = []
    c = _server_config(pim, keep, **over)
    handle = ctypes.c_void_p(1234)
    st = pim.lib.pim_server_create(ctypes.byref(c), ctypes.byref(handle))
    assert st == pim.PIM_ERR_INVALID
    assert frag in pim.lib.pim_last_error().decode()
    assert not handle.value


def test_server_calls_reject_null_handle(pim):
    import ctypes
    one = ctypes.c_int32()
    ids = np.zeros(1, np.uint32)
    ns = np.ones(1, np.int32)
    J = np.zeros((1, 1))
    jp = (ctypes.POINTER(ctypes.c_double) * 1)(J.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert pim.lib.pim_server_submit(None, 1, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                     ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), jp, None,
                                     ctypes.byref(one)) == pim.PIM_ERR_INVALID
    assert pim.lib.pim_server_flush(None, ctypes.byref(one)) == pim.PIM_ERR_INVALID
    assert pim.lib.pim_server_poll(None, 1, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None, None,
                                   ctypes.byref(one)) == pim.PIM_ERR_INVALID
    assert pim.lib.pim_server_pending(None, ctypes.byref(one), ctypes.byref(one)) == pim.PIM_ERR_INVALID
    pim.lib.pim_server_destroy(None)  # no-op


@pytest.mark.parametrize("J, h, what", [
    (np.array([[0, 200], [200, 0]]), None, "whole numbers"),      # would wrap in int8
    (np.array([[0, 0.5], [0.5, 0]]), None, "whole numbers"),
    (np.zeros((2, 3)), None, "square"),
    (np.zeros((3, 3)), np.zeros(2), "one entry per spin"),
    (np.zeros((2, 2)), np.array([2 ** 40, 0]), "int32 range"),
])
def test_instance_rejects_malformed_input_before_the_library(pim, J, h, what):
    """The binding refuses arrays that it could not hand over faithfully
    (values that a cast would change, shapes the library would read past)
    before any device call, so this runs without a GPU."""
    with pytest.raises(ValueError, match=what):
        pim.Instance(J, h, j_scale=1.0, xi=0.5)


def test_spin_arrays_refuse_values_the_cast_would_change(pim):
    """255 would become -1 in int8: the binding refuses it instead."""
    from paper_2604_17109_amd import _spins_int8
    assert _spins_int8(np.array([1, -1, 1.0])).dtype == np.int8
    with pytest.raises(ValueError, match="spins"):
        _spins_int8(np.array([1, 255]))


def test_mimo_helpers_check_shapes(pim):
    """Shapes that the library would read past are refused in the binding."""
    with pytest.raises(ValueError, match="square"):
        pim.quantize(np.zeros((2, 3)), "fp8")
    with pytest.raises(ValueError, match="H must be"):
        pim.mimo_ising(np.zeros((4, 2), complex), np.zeros(3, complex), 4, "ml")
    with pytest.raises(ValueError, match="spins"):
        pim.mimo_decode(np.zeros(4), np.ones(3), 4, "ml")       # 2 nt = 4 spins expected
    with pytest.raises(ValueError, match="spins"):
        pim.mimo_decode(np.zeros(4), np.ones(4), 16, "di")      # 4 nt = 8 spins expected
