"""pim_energy_noalloc (the entry point for callers that cannot allocate)
against pim_energy, through the C ABI: identical binary64 energies on two
calls in a row, the second with a smaller input, for integer and real-valued
instances, host and device spins; sizes beyond the fixed scratch array are
rejected before any device work."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def test_noalloc_energy_equals_pim_energy(gpu_lib):
    import torch
    pim = gpu_lib
    rng = np.random.default_rng(17)
    cases = []
    for n in (7, 200, 256):
        J, h = w.random_int8(n, seed=n, jmax=60 if n < 100 else 1, hmax=40)
        cases.append(pim.Instance(J, h, j_scale=0.01, xi=0.5))
    Jr = rng.standard_normal((96, 96))
    Jr = np.triu(Jr, 1)
    cases.append(pim.Instance(Jr + Jr.T, rng.standard_normal(96), j_scale=1.0, xi=2.0, prec="fp8"))
    for inst in cases:
        n = inst.n
        for count in (3000 if n < 100 else 900, 37):  # the second call is smaller
            _say(f"noalloc energy n={n} real={inst.real} count={count}")
            S = rng.choice(np.array([-1, 1], np.int8), size=(count, n))
            want = inst.energy(S)
            np.testing.assert_array_equal(inst.energy_noalloc(S), want)
            dev = torch.from_numpy(S).to("cuda")
            np.testing.assert_array_equal(inst.energy_noalloc(dev), want)
        inst.close()


def test_noalloc_rejects_sizes_beyond_scratch(gpu_lib):
    pim = gpu_lib
    n = 256
    J, h = w.sk1(n, seed=2)
    inst = pim.Instance(J, h, j_scale=1 / 16, xi=0.5)
    fits = (pim.NOALLOC_SCRATCH_BYTES - 8 * 4096) // n  # a count that fits with room to spare
    S = np.ones((fits, n), np.int8)
    _say(f"noalloc size limit n={n} count={fits}")
    np.testing.assert_array_equal(inst.energy_noalloc(S), inst.energy(S))
    too_many = np.ones((pim.NOALLOC_SCRATCH_BYTES // n + 1, n), np.int8)
    with pytest.raises(pim.PimError) as ei:
        inst.energy_noalloc(too_many)
    assert ei.value.status == pim.PIM_ERR_INVALID and "scratch" in str(ei.value)
    inst.close()
