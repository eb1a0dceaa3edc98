"""Plain, slow, CPU reference for the PIMI sweep and the conventional PIM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` do.  It shares no code with the HIP path; both
take their inputs from the ``workloads`` package.

Everything is NumPy in binary64 (integer fields in int64), one update step at a
time, in the paper's order and notation:

* Ising Hamiltonian, Eq. (1):  H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i.
* Local field, Eq. (2):        I_i(t) = sum_j J_ij s_j(t) + h_i.
* Conventional PIM, Eq. (3):   s_i(t+1) = sign[tanh(beta(t) I_i) + eta(t) U(-1,1)],
                               one spin i = t mod N per step (Box 1, top).
* PIMI, Eq. (4):               s_i(t+1) = sign[tanh(beta(t) I_i) + xi s_i(t)
                               + eta(t) N(0,1)], all spins at once (Box 1, bottom).
* tanh is the L-level lookup table of Suppl. "Quantization scheme",
  Algorithm "LUT-based tanh approximation".
* Couplings are normalised by a constant c (2/sqrt(N) for Max-Cut, 1/sqrt(N)
  for SK-1; Suppl. "Max-Cut instance generation" / "SK-1 instance generation",
  "Preprocessing"), applied after accumulation (Suppl. "Quantization scheme",
  Max-Cut and SK-1 paragraph).  The argument of tanh is (beta(t) * c) * I with the
  product beta(t) * c rounded first.

Readings where the paper is silent:
* sign(0): a tie keeps the current spin s_i(t).
* The LUT input x = 1 maps to the top level (half-open bins leave it unassigned).
* Noise: a B-bit uniform integer u from Philox4x32-10 keyed on (seed, trial,
  step, spin) selects Z[u] from a caller-supplied non-decreasing quantile table
  (Gaussian for PIMI, uniform for the conventional PIM).
"""
import numpy as np

from .philox import DOMAIN_INIT, DOMAIN_NOISE, uniform_bits


# ---------------------------------------------------------------------------
# Eq. (1) and Eq. (2)
# ---------------------------------------------------------------------------
def energy(J, h, s):
    """H(s) of Eq. (1) written as the double sum over i < j, exact in int64.

    ``s`` may be one configuration [N] or a batch [N, R] (one column per
    configuration); returns an int64 scalar or array [R].
    """
    J = np.asarray(J, dtype=np.int64)
    h = np.asarray(h, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    upper = np.triu(J, k=1)
    if s.ndim == 1:
        return -int(s @ upper @ s) - int(h @ s)
    pair = np.einsum("ir,ij,jr->r", s, upper, s)
    return -pair - h @ s


def energy_f64(J, h, s):
    """H(s) of Eq. (1) in binary64 for real-valued couplings (same double sum)."""
    J = np.asarray(J, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    upper = np.triu(J, k=1)
    if s.ndim == 1:
        return -float(s @ upper @ s) - float(h @ s)
    return -np.einsum("ir,ij,jr->r", s, upper, s) - h @ s


def energy_from_field(I, h, s):
    """E(s) = -1/2 sum_i s_i (I_i + h_i) with I = J s + h: the same value as
    Eq. (1) (J symmetric with zero diagonal), obtained from the field that the
    update computes anyway.  Exact in int64."""
    s = np.asarray(s, dtype=np.int64)
    h = np.asarray(h, dtype=np.int64)
    hb = h if s.ndim == 1 else h[:, None]
    twice = (s * (I + hb)).sum(axis=0)
    return -(twice // 2)


def local_field_f64(J, h, s):
    """I = J s + h of Eq. (2) for a real-valued instance, in binary64."""
    J = np.asarray(J, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    field = J @ s
    h = np.asarray(h, dtype=np.float64)
    return field + (h if field.ndim == 1 else h[:, None])


def energy_from_field_f64(I, h, s):
    """E(s) = -1/2 sum_i s_i (I_i + h_i) in binary64 (real-valued instance)."""
    s = np.asarray(s, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    hb = h if s.ndim == 1 else h[:, None]
    return -0.5 * (s * (I + hb)).sum(axis=0)


def local_field(J, h, s):
    """I = J s + h of Eq. (2), exact in int64 ([N] or [N, R])."""
    J = np.asarray(J, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    field = J @ s  # float64 matmul is exact for these integer magnitudes (< 2^53)
    field = np.rint(field).astype(np.int64)
    h = np.asarray(h, dtype=np.int64)
    return field + (h if field.ndim == 1 else h[:, None])


# ---------------------------------------------------------------------------
# Algorithm "LUT-based tanh approximation"
# ---------------------------------------------------------------------------
def lut_breakpoints(levels):
    """L + 1 uniformly spaced input breakpoints b_k = (2k - L) / L on [-1, 1]."""
    L = int(levels)
    return np.array([(2.0 * k - L) / L for k in range(L + 1)], dtype=np.float64)


def lut_levels(levels):
    """L uniformly spaced output levels (2k - (L-1)) / (L-1) on [-1, 1]."""
    L = int(levels)
    return np.array([(2.0 * k - (L - 1)) / (L - 1) for k in range(L)], dtype=np.float64)


def tanh_lut(x, levels):
    """L-level piecewise-constant tanh: saturate outside [-1, 1], otherwise the
    level of the bin [b_k, b_{k+1}) holding x (x = 1 gives the top level)."""
    L = int(levels)
    if L < 2:
        raise ValueError("a LUT needs at least two levels")
    x = np.asarray(x, dtype=np.float64)
    b = lut_breakpoints(L)
    lev = lut_levels(L)
    k = np.searchsorted(b, x, side="right") - 1  # b_k <= x < b_{k+1}
    k = np.clip(k, 0, L - 1)  # x >= 1 -> top bin; x < -1 -> bottom bin
    out = lev[k]
    out = np.where(x < -1.0, -1.0, out)
    out = np.where(x > 1.0, 1.0, out)
    return out


# ---------------------------------------------------------------------------
# One spin decision, Eq. (3) / Eq. (4)
# ---------------------------------------------------------------------------
def spin_decision(act, s, xi, eta, z):
    """sign[act + xi * s + eta * z] with a tie (exactly zero) keeping s.

    ``act`` is the already-evaluated tanh term.  Evaluation order is the
    paper's left to right: (act + xi*s) + eta*z, each operation rounded in
    binary64.
    """
    s = np.asarray(s, dtype=np.int64)
    v = (act + xi * s) + eta * z
    return np.where(v > 0, 1, np.where(v < 0, -1, s)).astype(np.int64)


def initial_spins(seed, stream, trials, n, bits=8):
    """s_i(0) = +1 if u >= 2^(B-1) else -1, with u from the INIT counter domain
    at step 0.  Returns int64 [n, trials]."""
    spin = np.arange(n)[:, None]
    trial = np.asarray(trials)[None, :]
    u = uniform_bits(seed, DOMAIN_INIT, stream, trial, 0, spin, bits)
    return np.where(u >= (1 << (bits - 1)), 1, -1).astype(np.int64)


class Problem:
    """An integer Ising instance plus the update-rule constants.

    J: symmetric int matrix with zero diagonal; h: int vector; c: coupling
    normalisation; xi: inertia (0 for the conventional PIM); levels: L;
    ztab: non-decreasing float64 quantile table of length 2^bits.
    """
    real = False

    def __init__(self, J, h, c, xi, levels, ztab, bits=8):
        self.J = np.asarray(J, dtype=np.int64)
        self.h = np.asarray(h, dtype=np.int64)
        self.n = self.J.shape[0]
        if self.J.shape != (self.n, self.n) or self.h.shape != (self.n,):
            raise ValueError("J must be N x N and h length N")
        if not np.array_equal(self.J, self.J.T) or np.any(np.diag(self.J) != 0):
            raise ValueError("J must be symmetric with a zero diagonal")
        self.c = float(c)
        self.xi = float(xi)
        self.levels = int(levels)
        self.ztab = np.asarray(ztab, dtype=np.float64)
        self.bits = int(bits)
        if self.ztab.shape != (1 << self.bits,):
            raise ValueError("noise table length must be 2^bits")


class RealProblem(Problem):
    """A real-valued Ising instance (binary64 J and h; e.g. the MIMO detection
    instances of Suppl. "Delta-Ising MIMO (DI-MIMO) formulation") with the same
    update-rule constants.  Fields and energies are binary64; the update rule is
    unchanged (the LUT argument is (beta(t) * c) * I with I in binary64)."""
    real = True

    def __init__(self, J, h, c, xi, levels, ztab, bits=8):
        self.J = np.asarray(J, dtype=np.float64)
        self.h = np.asarray(h, dtype=np.float64)
        self.n = self.J.shape[0]
        if self.J.shape != (self.n, self.n) or self.h.shape != (self.n,):
            raise ValueError("J must be N x N and h length N")
        if not np.array_equal(self.J, self.J.T) or np.any(np.diag(self.J) != 0):
            raise ValueError("J must be symmetric with a zero diagonal")
        if not (np.all(np.isfinite(self.J)) and np.all(np.isfinite(self.h))):
            raise ValueError("J and h must be finite")
        self.c = float(c)
        self.xi = float(xi)
        self.levels = int(levels)
        self.ztab = np.asarray(ztab, dtype=np.float64)
        self.bits = int(bits)
        if self.ztab.shape != (1 << self.bits,):
            raise ValueError("noise table length must be 2^bits")


def _result(n_trials, n, real=False):
    return {
        "e_best": np.full(n_trials, np.inf) if real else np.full(n_trials, np.iinfo(np.int64).max, dtype=np.int64),
        "t_best": np.full(n_trials, -1, dtype=np.int64),
        "best_state": np.zeros((n, n_trials), dtype=np.int64),
        "first_hit": np.full(n_trials, -1, dtype=np.int64),
    }


def _track(res, e, s, t, target):
    better = e < res["e_best"]  # strict: ties keep the earliest step
    res["e_best"] = np.where(better, e, res["e_best"])
    res["t_best"] = np.where(better, t, res["t_best"])
    res["best_state"][:, better] = s[:, better]
    if target is not None:
        hit = (e <= target) & (res["first_hit"] < 0)
        res["first_hit"] = np.where(hit, t, res["first_hit"])


def _noise_values(prob, seed, stream, trials, step, spin, noise):
    if noise is None:
        u = uniform_bits(seed, DOMAIN_NOISE, stream, trials, step, spin, prob.bits)
        return prob.ztab[u]
    return noise(np.broadcast_shapes(np.shape(spin), np.shape(trials)), step)


def _activation(prob, x, act):
    return tanh_lut(x, prob.levels) if act is None else act(x)


def run_parallel(prob, beta, eta, seed, stream, trials, init=None, start_step=0,
                 target=None, trace=False, act=None, noise=None, record=False):
    """PIMI (Eq. (4), Box 1): every spin of every trial updated at each step.

    ``beta``, ``eta``: float64 arrays of length T (step t uses index t).  The
    noise of step t of trial a for spin i comes from counter step
    start_step + t.  Trials are the integer ids in ``trials``.

    Returns final spins s(T) [N, R] and, over the energies E(t) of s(t) for
    t = 0..T (global index start_step + t): the lowest energy, its earliest
    step, the state there, and the first step with E <= target.

    ``act`` (default: the L-level LUT) and ``noise`` (default: Philox index into
    the quantile table; otherwise ``noise(shape, step) -> float64 array``) are
    overridable so that statistical pins can run the same loop with the exact
    tanh and continuous noise.  ``record`` keeps every state: res["states"] is
    int8 [T + 1, N, R] with s(t) at index t.
    """
    beta = np.asarray(beta, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    steps = len(beta)
    trials = np.asarray(trials, dtype=np.int64)
    n = prob.n
    s = initial_spins(seed, stream, trials, n, prob.bits) if init is None \
        else np.asarray(init, dtype=np.int64).copy()
    res = _result(len(trials), n, prob.real)
    energies = []
    states = []
    spin = np.arange(n)[:, None]
    for t in range(steps + 1):
        if record:
            states.append(s.astype(np.int8))
        if prob.real:
            I = local_field_f64(prob.J, prob.h, s)
            e = energy_from_field_f64(I, prob.h, s)
        else:
            I = local_field(prob.J, prob.h, s)
            e = energy_from_field(I, prob.h, s)
        _track(res, e, s, start_step + t, target)
        if trace:
            energies.append(e)
        if t == steps:
            break
        g = beta[t] * prob.c
        a = _activation(prob, g * I, act)
        z = _noise_values(prob, seed, stream, trials[None, :], start_step + t, spin, noise)
        s = spin_decision(a, s, prob.xi, eta[t], z)
    res["final"] = s
    if trace:
        res["trace"] = np.stack(energies, axis=0)
    if record:
        res["states"] = np.stack(states, axis=0)
    return res


def run_sequential(prob, beta, eta, seed, stream, trials, init=None, start_step=0,
                   target=None, trace=False, act=None, noise=None):
    """Conventional PIM with sequential updates (Eq. (3), Box 1 top): at step t
    only spin i = t mod N changes, using the local field of the current
    configuration and the noise value of (trial, step t, spin i)."""
    beta = np.asarray(beta, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    steps = len(beta)
    trials = np.asarray(trials, dtype=np.int64)
    n = prob.n
    s = initial_spins(seed, stream, trials, n, prob.bits) if init is None \
        else np.asarray(init, dtype=np.int64).copy()
    res = _result(len(trials), n, prob.real)
    energies = []
    for t in range(steps + 1):
        e = energy_f64(prob.J, prob.h, s) if prob.real else energy(prob.J, prob.h, s)
        _track(res, e, s, start_step + t, target)
        if trace:
            energies.append(e)
        if t == steps:
            break
        tg = start_step + t
        i = tg % n
        I_i = (prob.J[i].astype(np.float64) @ s.astype(np.float64) + prob.h[i]) if prob.real \
            else prob.J[i] @ s + prob.h[i]
        a = _activation(prob, (beta[t] * prob.c) * I_i, act)
        z = _noise_values(prob, seed, stream, trials, tg, i, noise)
        s = s.copy()
        s[i] = spin_decision(a, s[i], prob.xi, eta[t], z)
    res["final"] = s
    if trace:
        res["trace"] = np.stack(energies, axis=0)
    return res
