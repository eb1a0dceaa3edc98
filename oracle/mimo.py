"""Plain CPU reference of MIMO detection as an Ising problem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` do.  It shares no code with the HIP path.

Everything is NumPy binary64, written from the paper's definitions:

* real-valued equivalent of the complex model (Suppl. "Real-Valued
  equivalent"): H -> [[Re H, -Im H], [Im H, Re H]], y -> [Re y; Im y];
* the linear MMSE detector with hard slicing (Suppl. "Baseline: linear MMSE
  detector"): z = (H^H H + (1 / (Es/N0)) I)^-1 H^H y, then each component is
  sliced to the nearest constellation level;
* the perturbation mapping (Suppl. "Delta-Ising MIMO (DI-MIMO) formulation"):
  x = x_m + T s with s in {-1, +1}^K, and the Ising parameters
  J_DI = -zeroDiag(T^T H^T H T), h = 2 T^T H^T (y - H x_m), whose objective
  -h^T s - s^T J_DI s equals ||y - H(x_m + T s)||^2 up to a constant;
* reconstruction x = slice(x_m + T s) and the bit / symbol error rates (Suppl.
  "Performance metric: bit-error rate (BER)").

Readings where the paper is silent:
* The Ising instance handed to the solver uses the Eq. (1) convention
  H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i, so its couplings are
  J = 2 J_DI (every pair appears once in Eq. (1) but twice in s^T J_DI s) and
  its local field I = J s + h is the exact negative gradient of the residual.
* Two mappings: "ml" (x_m = 0, T = I for 4-QAM and T = [2I, I] for 16-QAM, so
  x = T s spans the constellation exactly) and "di" (x_m = the sliced MMSE
  estimate, T = [I, I], corrections D = {-2, 0, 2} per real component).
* Slicing maps v to the odd integer 2 floor(v / 2) + 1 clipped to the
  constellation (a value exactly on an even integer goes up).
"""
import itertools

import numpy as np


def real_equivalent(Hc, yc):
    """(H [2Nr, 2Nt], y [2Nr]) of the real-valued model."""
    Hc = np.asarray(Hc, dtype=np.complex128)
    yc = np.asarray(yc, dtype=np.complex128)
    H = np.block([[Hc.real, -Hc.imag], [Hc.imag, Hc.real]])
    return H, np.concatenate([yc.real, yc.imag])


def real_vector(xc):
    xc = np.asarray(xc, dtype=np.complex128)
    return np.concatenate([xc.real, xc.imag])


def complex_vector(xr):
    xr = np.asarray(xr, dtype=np.float64)
    n = xr.shape[0] // 2
    return xr[:n] + 1j * xr[n:]


def slice_levels(v, qam):
    """Nearest level of the sqrt(M)-level odd-integer alphabet, per component."""
    m = int(round(np.sqrt(qam)))
    v = np.asarray(v, dtype=np.float64)
    return np.clip(2.0 * np.floor(v / 2.0) + 1.0, -(m - 1), m - 1)


def mmse(Hc, yc, esn0):
    """Unsliced linear MMSE estimate z (complex [Nt]) with the paper's
    regulariser 1 / (Es/N0)."""
    Hc = np.asarray(Hc, dtype=np.complex128)
    A = Hc.conj().T @ Hc + (1.0 / esn0) * np.eye(Hc.shape[1])
    return np.linalg.solve(A, Hc.conj().T @ np.asarray(yc, dtype=np.complex128))


def mmse_detect(Hc, yc, esn0, qam):
    z = mmse(Hc, yc, esn0)
    return slice_levels(z.real, qam) + 1j * slice_levels(z.imag, qam)


def transform_weights(mode, qam):
    """Block weights w of T = [w_0 I, w_1 I, ...] for a mapping."""
    if mode == "ml":
        if qam == 4:
            return [1.0]
        if qam == 16:
            return [2.0, 1.0]
        raise ValueError("the 'ml' mapping covers 4-QAM and 16-QAM")
    if mode == "di":
        return [1.0, 1.0]
    raise ValueError(f"unknown mapping {mode!r}")


def transform(mode, qam, n2):
    return np.hstack([w * np.eye(n2) for w in transform_weights(mode, qam)])


def ising(H, y, xm, T):
    """(J, h, const) with ||y - H(xm + T s)||^2 = E_Eq1(s; J, h) + const."""
    r = y - H @ xm
    G = T.T @ H.T @ H @ T
    J = -2.0 * (G - np.diag(np.diag(G)))
    h = 2.0 * (T.T @ (H.T @ r))
    return J, h, float(r @ r + np.trace(G))


def detector_instance(problem, mode):
    """Ising instance of one workloads.mimo problem: dict with J, h, xm, T, const."""
    H, y = real_equivalent(problem["H"], problem["y"])
    n2 = H.shape[1]
    if mode == "ml":
        xm = np.zeros(n2)
    else:
        xm = real_vector(mmse_detect(problem["H"], problem["y"], problem["esn0"], problem["qam"]))
    T = transform(mode, problem["qam"], n2)
    J, h, const = ising(H, y, xm, T)
    return {"J": J, "h": h, "xm": xm, "T": T, "const": const, "H": H, "y": y}


def decode(xm, T, s, qam):
    """Detected complex symbols from a spin vector s [K] (or [K, R])."""
    s = np.asarray(s, dtype=np.float64)
    x = (xm if s.ndim == 1 else xm[:, None]) + T @ s
    x = slice_levels(x, qam)
    n = x.shape[0] // 2
    return x[:n] + 1j * x[n:]


def ml_enumerate(Hc, yc, qam):
    """Exact ML detection by enumerating every symbol vector (small Nt only)."""
    from workloads.mimo import pam_levels  # the alphabet is part of the input's definition
    Hc = np.asarray(Hc, dtype=np.complex128)
    nt = Hc.shape[1]
    lv = pam_levels(qam).astype(np.float64)
    pts = np.array([a + 1j * b for a in lv for b in lv])
    best, arg = np.inf, None
    for combo in itertools.product(range(len(pts)), repeat=nt):
        x = pts[list(combo)]
        d = np.linalg.norm(yc - Hc @ x) ** 2
        if d < best:
            best, arg = d, x
    return arg, best


def symbol_errors(x_tx, x_rx):
    return int(np.count_nonzero(np.asarray(x_tx) != np.asarray(x_rx)))


def bit_errors(bits_tx, bits_rx):
    return int(np.count_nonzero(np.asarray(bits_tx) != np.asarray(bits_rx)))
