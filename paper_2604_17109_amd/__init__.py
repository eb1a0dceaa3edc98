"""Python binding of libpim.so, the MI355X PIMI sweep library.

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch supplies the device allocator (its caching allocator) and
the stream (its current stream); nothing here computes the method.

    import paper_2604_17109_amd as pim
    inst = pim.Instance(J, h, j_scale=1/np.sqrt(n), xi=0.5, levels=4)
    batch = pim.Batch([inst], trials=1024)
    batch.run(beta, eta, seed=1)
    spins, energy, trial, step = batch.best(0)

The library refuses to fall back to anything else: if libpim.so is missing
the import raises.
"""
import ctypes
import os

import numpy as np
# torch first: its HIP runtime must be the one libpim.so binds to, or a
# process that loads the library before touching torch ends up with two
# runtimes and the library's sees no device
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpim.so")

PIM_OK, PIM_ERR_INVALID, PIM_ERR_UNSUPPORTED, PIM_ERR_NOMEM = 0, 1, 2, 3
PIM_ERR_DEVICE, PIM_ERR_STATE, PIM_ERR_CANCELLED = 4, 5, 6
NOISE_GAUSS, NOISE_UNIFORM = 0, 1
KERNEL_MFMA_I8, KERNEL_PLAIN_F32, KERNEL_SEQ_I8, KERNEL_MFMA_F4 = 0, 1, 2, 3
PREC_FP8, PREC_BF16 = 1, 2
MIMO_ML, MIMO_DI = 0, 1
ABI_VERSION = 2
_PRECS = {"fp8": PREC_FP8, "bf16": PREC_BF16}
_MAPS = {"ml": MIMO_ML, "di": MIMO_DI}
_KERNELS = {"mfma": KERNEL_MFMA_I8, "mfma_i8": KERNEL_MFMA_I8, "plain": KERNEL_PLAIN_F32,
            "plain_f32": KERNEL_PLAIN_F32, "seq": KERNEL_SEQ_I8, "sequential": KERNEL_SEQ_I8,
            "mfma_f4": KERNEL_MFMA_F4, "f4": KERNEL_MFMA_F4}
_NOISES = {"gauss": NOISE_GAUSS, "uniform": NOISE_UNIFORM}

# every symbol declared in include/pim.h
EXPORTED = (
    "pim_set_allocator", "pim_create", "pim_batch_create", "pim_run", "pim_cancel",
    "pim_energy", "pim_best", "pim_trials", "pim_kernel_time", "pim_compile_step", "pim_compile_table",
    "pim_batch_destroy", "pim_destroy", "pim_last_error", "pim_abi_version",
    "pim_create_real", "pim_quantize", "pim_compile_table_real", "pim_mimo_ising", "pim_mimo_decode",
    "pim_states", "pim_flip_counts", "pim_tune",
    "pim_server_create", "pim_server_submit", "pim_server_flush", "pim_server_poll", "pim_server_pending",
    "pim_server_destroy", "pim_energy_noalloc", "pim_server_poll_times",
    "pim_mimo_ising_device", "pim_server_create_mimo", "pim_server_submit_mimo", "pim_server_poll_mimo",
)
MAX_N_LDS = 256
NOALLOC_SCRATCH_BYTES = 1 << 20


class PimError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[pim status {status}] {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("j_scale", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("levels", ctypes.c_int32),
        ("noise", ctypes.c_int32),
        ("noise_bits", ctypes.c_int32),
        ("noise_table", ctypes.POINTER(ctypes.c_double)),
        ("rng_stream", ctypes.c_uint32),
    ]


class Schedule(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("eta", ctypes.POINTER(ctypes.c_double)),
        ("start_step", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("use_target", ctypes.c_int32),
        ("target", ctypes.POINTER(ctypes.c_double)),
        ("record_states", ctypes.c_int32),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("max_n", ctypes.c_int32),
        ("slots_per_class", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("trials", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("eta", ctypes.POINTER(ctypes.c_double)),
        ("j_scale", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("levels", ctypes.c_int32),
        ("noise", ctypes.c_int32),
        ("noise_table", ctypes.POINTER(ctypes.c_double)),
        ("prec", ctypes.c_int32),
        ("streams", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("hbm_budget", ctypes.c_size_t),
        ("max_wait_us", ctypes.c_double),
        ("prealloc_chunks", ctypes.c_int32),
    ]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2604_17109_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, F64, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    sig = {
        "pim_set_allocator": (I32, [_ALLOC_FN, _FREE_FN, VP]),
        "pim_create": (I32, [P(ctypes.c_int8), P(ctypes.c_int32), P(Params), VP, P(VP)]),
        "pim_batch_create": (I32, [P(VP), I32, I32, P(ctypes.c_int8), VP, P(VP)]),
        "pim_run": (I32, [VP, P(Schedule), ctypes.c_uint64, VP]),
        "pim_cancel": (I32, [VP]),
        "pim_energy": (I32, [VP, P(ctypes.c_int8), I32, P(F64), VP]),
        "pim_energy_noalloc": (I32, [VP, P(ctypes.c_int8), I32, P(F64), VP]),
        "pim_best": (I32, [VP, I32, P(ctypes.c_int8), P(F64), P(I32), P(I32)]),
        "pim_trials": (I32, [VP, I32, P(F64), P(I32), P(I32), P(F64), P(ctypes.c_int8), P(ctypes.c_int8)]),
        "pim_kernel_time": (I32, [VP, P(ctypes.c_float)]),
        "pim_compile_step": (I32, [P(Params), F64, F64, P(I32), P(I32)]),
        "pim_compile_table": (I32, [P(Params), F64, F64, P(ctypes.c_int16)]),
        "pim_batch_destroy": (None, [VP]),
        "pim_destroy": (None, [VP]),
        "pim_last_error": (ctypes.c_char_p, []),
        "pim_abi_version": (I32, []),
        "pim_create_real": (I32, [P(F64), P(F64), P(Params), I32, VP, P(VP)]),
        "pim_quantize": (I32, [P(F64), I32, I32, P(F64), P(F64)]),
        "pim_compile_table_real": (I32, [P(Params), F64, F64, P(ctypes.c_float)]),
        "pim_mimo_ising": (I32, [P(F64), P(F64), I32, I32, I32, I32, F64, P(F64), P(F64), P(F64), P(I32)]),
        "pim_mimo_decode": (I32, [P(F64), P(ctypes.c_int8), I32, I32, I32, P(F64)]),
        "pim_states": (I32, [VP, I32, I32, P(ctypes.c_int8)]),
        "pim_flip_counts": (I32, [VP, I32, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "pim_tune": (I32, [VP, I32, VP, P(I32)]),
        "pim_server_create": (I32, [P(ServerConfig), P(VP)]),
        # ids, ns and the two pointer tables go as raw addresses of numpy arrays
        "pim_server_submit": (I32, [VP, I32, VP, VP, VP, VP, P(I32)]),
        "pim_server_flush": (I32, [VP, P(I32)]),
        "pim_server_poll": (I32, [VP, I32, P(ctypes.c_uint32), P(ctypes.c_int8), P(F64), P(I32)]),
        "pim_server_pending": (I32, [VP, P(I32), P(I32)]),
        "pim_server_poll_times": (I32, [VP, I32, P(ctypes.c_uint32), P(ctypes.c_int8), P(F64), P(F64), P(I32)]),
        "pim_mimo_ising_device": (I32, [P(F64), P(F64), I32, I32, I32, I32, F64, P(F64), P(F64), P(F64), P(I32),
                                        VP]),
        "pim_server_create_mimo": (I32, [P(ServerConfig), P(VP)]),
        # ids, dims, esn0 and the two pointer tables go as raw addresses of numpy arrays
        "pim_server_submit_mimo": (I32, [VP, I32, VP, VP, VP, VP, VP, P(I32)]),
        "pim_server_poll_mimo": (I32, [VP, I32, P(ctypes.c_uint32), P(ctypes.c_int8), P(F64), P(F64), P(F64),
                                       P(I32)]),
        "pim_server_destroy": (None, [VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.pim_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} implements ABI {lib.pim_abi_version()}, this binding needs {ABI_VERSION}; "
                          "rebuild with `python paper_2604_17109_amd/build.py`")
    return lib


lib = _load()


def _check(status):
    if status != PIM_OK:
        raise PimError(status, lib.pim_last_error().decode(errors="replace"))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


# ---------------------------------------------------------------------------
# torch plumbing: caching allocator and current stream
# ---------------------------------------------------------------------------
_torch_hooks = None


def use_torch_allocator():
    """Route every device allocation of the library through torch's caching
    allocator (idempotent)."""
    global _torch_hooks
    if _torch_hooks is not None:
        return
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
        except Exception:  # noqa: BLE001 - reported to the library as NULL (PIM_ERR_NOMEM)
            return None

    def _free(ptr, stream, user):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib.pim_set_allocator(hooks[0], hooks[1], None))
    _torch_hooks = hooks


def current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _device_ready():
    import torch
    if not torch.cuda.is_available():
        raise PimError(PIM_ERR_DEVICE, "no GPU visible to torch")
    use_torch_allocator()


# ---------------------------------------------------------------------------
def make_params(n, j_scale, xi, levels=4, noise="gauss", noise_table=None, rng_stream=0,
                noise_bits=8):
    p = Params()
    p.n = int(n)
    p.j_scale = float(j_scale)
    p.xi = float(xi)
    p.levels = int(levels)
    p.noise = _NOISES[noise] if isinstance(noise, str) else int(noise)
    p.noise_bits = int(noise_bits)
    keep = None
    if noise_table is not None:
        keep = np.ascontiguousarray(noise_table, dtype=np.float64)
        p.noise_table = _ptr(keep, ctypes.c_double)
    p.rng_stream = int(rng_stream)
    return p, keep


def validate(J, h=None, *, j_scale, xi, levels=4, noise="gauss", noise_table=None, noise_bits=8, prec=None):
    """Runs pim_create's (``prec`` None) or pim_create_real's argument
    validation only (no device work): returns None when the arguments are
    valid, else raises PimError.  Valid input is detected by the library
    reaching its first device allocation, which this call forbids through a
    refusing allocator."""
    real = prec is not None
    J = np.ascontiguousarray(J, dtype=np.float64 if real else np.int8)
    if h is None:
        hh = None
    else:
        hh = np.ascontiguousarray(h, dtype=np.float64 if real else np.int32)
    p, keep = make_params(J.shape[0] if J.ndim == 2 else 0, j_scale, xi, levels, noise, noise_table,
                          noise_bits=noise_bits)
    handle = ctypes.c_void_p()
    refuse = (_ALLOC_FN(lambda nb, st, u: None), _FREE_FN(lambda ptr, st, u: None))
    prev = _torch_hooks
    _check(lib.pim_set_allocator(refuse[0], refuse[1], None))
    try:
        if real:
            st = lib.pim_create_real(_ptr(J, ctypes.c_double), _ptr(hh, ctypes.c_double), ctypes.byref(p),
                                     _PRECS.get(prec, -1) if isinstance(prec, str) else int(prec), None,
                                     ctypes.byref(handle))
        else:
            st = lib.pim_create(_ptr(J, ctypes.c_int8), _ptr(hh, ctypes.c_int32), ctypes.byref(p), None,
                                ctypes.byref(handle))
    finally:
        if prev is not None:
            _check(lib.pim_set_allocator(prev[0], prev[1], None))
        else:
            _check(lib.pim_set_allocator(_ALLOC_FN(0), _FREE_FN(0), None))
    del keep
    if st == PIM_ERR_NOMEM:
        return None  # validation passed; the refusing allocator stopped it
    _check(st)
    lib.pim_destroy(handle)
    return None


def compile_step(n, j_scale, xi, beta, eta, levels=4, noise="gauss", noise_table=None):
    """Host-only: integer thresholds (theta[L-1], umin[2L]) compiled for one step."""
    p, keep = make_params(n, j_scale, xi, levels, noise, noise_table)
    theta = np.zeros(levels - 1, dtype=np.int32)
    umin = np.zeros(2 * levels, dtype=np.int32)
    _check(lib.pim_compile_step(ctypes.byref(p), float(beta), float(eta), _ptr(theta, ctypes.c_int32),
                                _ptr(umin, ctypes.c_int32)))
    del keep
    return theta, umin


def compile_table(n, j_scale, xi, beta, eta, levels=4, noise="gauss", noise_table=None):
    """Host-only: the 512-entry (u, s) field-threshold table of one step."""
    p, keep = make_params(n, j_scale, xi, levels, noise, noise_table)
    tab = np.zeros(512, dtype=np.int16)
    _check(lib.pim_compile_table(ctypes.byref(p), float(beta), float(eta), _ptr(tab, ctypes.c_int16)))
    del keep
    return tab


def compile_table_real(n, j_scale, xi, beta, eta, levels=4, noise="gauss", noise_table=None):
    """Host-only: the 512-entry (u, s) binary32 field-threshold table of one
    step for real-valued instances."""
    p, keep = make_params(n, j_scale, xi, levels, noise, noise_table)
    tab = np.zeros(512, dtype=np.float32)
    _check(lib.pim_compile_table_real(ctypes.byref(p), float(beta), float(eta), _ptr(tab, ctypes.c_float)))
    del keep
    return tab


def quantize(J, prec):
    """Host-only: (couplings scale * q as float64, scale) that the batched kernel
    uses for a real-valued J in precision "fp8" or "bf16"."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    if J.ndim != 2 or J.shape[0] != J.shape[1]:
        raise ValueError("J must be square")
    out = np.zeros_like(J)
    scale = ctypes.c_double()
    _check(lib.pim_quantize(_ptr(J, ctypes.c_double), J.shape[0], _PRECS[prec], _ptr(out, ctypes.c_double),
                            ctypes.byref(scale)))
    return out, scale.value


def _complex_interleaved(z):
    z = np.asarray(z, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1))


def mimo_ising(H, y, qam, mapping="di", esn0=1.0):
    """Ising instance of one MIMO detection problem y = H x + n (complex H
    [nr, nt], y [nr]): returns (J [n, n], h [n], x_m [2 nt]), all float64."""
    Hc = _complex_interleaved(H)
    yc = _complex_interleaved(y)
    if Hc.ndim != 3 or yc.shape != (Hc.shape[0], 2):
        raise ValueError("H must be [nr, nt] and y [nr]")
    nr, nt = Hc.shape[0], Hc.shape[1]
    J = np.zeros((4 * nt, 4 * nt), np.float64)
    h = np.zeros(4 * nt, np.float64)
    xm = np.zeros(2 * nt, np.float64)
    n = ctypes.c_int32()
    _check(lib.pim_mimo_ising(_ptr(Hc, ctypes.c_double), _ptr(yc, ctypes.c_double), nr, nt, int(qam),
                              _MAPS[mapping], float(esn0), _ptr(J, ctypes.c_double), _ptr(h, ctypes.c_double),
                              _ptr(xm, ctypes.c_double), ctypes.byref(n)))
    k = n.value
    # the library writes J as a dense k x k block at the start of the buffer
    return np.ascontiguousarray(J.reshape(-1)[: k * k].reshape(k, k)), h[:k].copy(), xm


def mimo_ising_device(H, y, qam, mapping="di", esn0=1.0, stream=None):
    """mimo_ising computed by the device mapping kernel (binary64)."""
    Hc = _complex_interleaved(H)
    yc = _complex_interleaved(y)
    if Hc.ndim != 3 or yc.shape != (Hc.shape[0], 2):
        raise ValueError("H must be [nr, nt] and y [nr]")
    nr, nt = Hc.shape[0], Hc.shape[1]
    J = np.zeros((4 * nt, 4 * nt), np.float64)
    h = np.zeros(4 * nt, np.float64)
    xm = np.zeros(2 * nt, np.float64)
    n = ctypes.c_int32()
    _device_ready()
    _check(lib.pim_mimo_ising_device(_ptr(Hc, ctypes.c_double), _ptr(yc, ctypes.c_double), nr, nt, int(qam),
                                     _MAPS[mapping], float(esn0), _ptr(J, ctypes.c_double), _ptr(h, ctypes.c_double),
                                     _ptr(xm, ctypes.c_double), ctypes.byref(n),
                                     stream if stream is not None else current_stream()))
    k = n.value
    return np.ascontiguousarray(J.reshape(-1)[: k * k].reshape(k, k)), h[:k].copy(), xm


def mimo_decode(xm, spins, qam, mapping="di"):
    """Detected complex symbols [nt] of a spin vector under the same mapping."""
    xm = np.ascontiguousarray(xm, dtype=np.float64)
    s = _spins_int8(spins)
    nt = xm.size // 2
    n = 2 * nt if (mapping == "ml" and int(qam) == 4) else 4 * nt
    if xm.size != 2 * nt or int(qam) not in (4, 16) or s.size != n:
        raise ValueError("x_m must be [2 nt] and spins [2 nt] (ML, 4-QAM) or [4 nt]")
    x = np.zeros((nt, 2), np.float64)
    _check(lib.pim_mimo_decode(_ptr(xm, ctypes.c_double), _ptr(s, ctypes.c_int8), nt, int(qam), _MAPS[mapping],
                               _ptr(x, ctypes.c_double)))
    return x[:, 0] + 1j * x[:, 1]


def _spins_int8(a):
    """a as contiguous int8, refusing values that the cast would change."""
    a_in = np.asarray(a)
    s = np.ascontiguousarray(a_in, dtype=np.int8)
    if not np.array_equal(s, a_in):
        raise ValueError("spins must be +1 or -1")
    return s


class Instance:
    """One Ising instance with its update-rule constants, copied to the device.

    Integer instance (default): J int8 symmetric with zero diagonal, h int32.
    Real-valued instance (``prec`` = "fp8" or "bf16"): J, h float64; the batched
    kernel uses J quantised to ``prec`` with a per-instance scale."""

    def __init__(self, J, h=None, *, j_scale, xi, levels=4, noise="gauss", noise_table=None,
                 rng_stream=0, prec=None, stream=None):
        self.real = prec is not None
        Jin = np.asarray(J)
        J = np.ascontiguousarray(Jin, dtype=np.float64 if self.real else np.int8)
        if J.ndim != 2 or J.shape[0] != J.shape[1]:
            raise ValueError("J must be square")
        if not self.real and not np.array_equal(J, Jin):
            raise ValueError("integer couplings must be whole numbers in [-128, 127]")
        self.n = J.shape[0]
        if h is not None:
            hin = np.asarray(h)
            if hin.shape != (self.n,):
                raise ValueError("h must have one entry per spin")
            if not self.real and not np.array_equal(hin.astype(np.int32), hin):
                raise ValueError("integer fields must be whole numbers in the int32 range")
        p, keep = make_params(self.n, j_scale, xi, levels, noise, noise_table, rng_stream)
        self._handle = ctypes.c_void_p()
        _device_ready()
        st = stream if stream is not None else current_stream()
        if self.real:
            hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
            _check(lib.pim_create_real(_ptr(J, ctypes.c_double), _ptr(hh, ctypes.c_double), ctypes.byref(p),
                                       _PRECS[prec], st, ctypes.byref(self._handle)))
        else:
            hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
            _check(lib.pim_create(_ptr(J, ctypes.c_int8), _ptr(hh, ctypes.c_int32), ctypes.byref(p), st,
                                  ctypes.byref(self._handle)))
        del keep

    @property
    def handle(self):
        return self._handle

    def energy(self, spins, stream=None):
        """Binary64 energies (Eq. (1)) of configurations spins[count, n]: a
        host array, or a contiguous int8 torch tensor on the GPU, which the
        library reads in place (its values are not checked: they must be
        +-1)."""
        import torch
        if isinstance(spins, torch.Tensor) and spins.is_cuda:
            if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != self.n \
                    or not spins.is_contiguous() or spins.shape[0] < 1:
                raise ValueError("device spins must be a contiguous int8 tensor [count, n]")
            out = np.zeros(spins.shape[0], dtype=np.float64)
            _check(lib.pim_energy(self._handle, ctypes.cast(ctypes.c_void_p(spins.data_ptr()),
                                                            ctypes.POINTER(ctypes.c_int8)),
                                  spins.shape[0], _ptr(out, ctypes.c_double),
                                  stream if stream is not None else current_stream()))
            return out
        s = _spins_int8(np.atleast_2d(spins))
        if s.ndim != 2 or s.shape[1] != self.n:
            raise ValueError("spins must be [count, n]")
        out = np.zeros(s.shape[0], dtype=np.float64)
        _check(lib.pim_energy(self._handle, _ptr(s, ctypes.c_int8), s.shape[0], _ptr(out, ctypes.c_double),
                              stream if stream is not None else current_stream()))
        return out

    def energy_noalloc(self, spins, stream=None):
        """energy() through pim_energy_noalloc: no device allocation (the
        library's fixed per-GPU scratch array holds the staging)."""
        import torch
        st = stream if stream is not None else current_stream()
        if isinstance(spins, torch.Tensor) and spins.is_cuda:
            if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != self.n \
                    or not spins.is_contiguous() or spins.shape[0] < 1:
                raise ValueError("device spins must be a contiguous int8 tensor [count, n]")
            out = np.zeros(spins.shape[0], dtype=np.float64)
            _check(lib.pim_energy_noalloc(self._handle, ctypes.cast(ctypes.c_void_p(spins.data_ptr()),
                                                                    ctypes.POINTER(ctypes.c_int8)),
                                          spins.shape[0], _ptr(out, ctypes.c_double), st))
            return out
        s = _spins_int8(np.atleast_2d(spins))
        if s.ndim != 2 or s.shape[1] != self.n:
            raise ValueError("spins must be [count, n]")
        out = np.zeros(s.shape[0], dtype=np.float64)
        _check(lib.pim_energy_noalloc(self._handle, _ptr(s, ctypes.c_int8), s.shape[0],
                                      _ptr(out, ctypes.c_double), st))
        return out

    def close(self):
        if self._handle:
            lib.pim_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Batch:
    """Instances x `trials` trials, with per-trial result buffers.  Instances
    of different N run together (one graph launch per run)."""

    def __init__(self, instances, trials, init_spins=None, stream=None):
        _device_ready()
        self.instances = list(instances)  # keep the instances alive
        self.count = len(self.instances)
        self.trials = int(trials)
        self.ns = [i.n for i in self.instances]
        self.n = self.ns[0] if len(set(self.ns)) == 1 else None
        arr = (ctypes.c_void_p * self.count)(*[i.handle.value for i in self.instances])
        init = None
        if init_spins is not None:
            if self.n is not None:
                init = _spins_int8(init_spins).reshape(self.count, self.trials, self.n)
            else:  # a sequence of [trials, n_k] arrays
                parts = list(init_spins)
                if len(parts) != self.count:
                    raise ValueError("init_spins needs one [trials, n_k] array per instance")
                for a, n in zip(parts, self.ns):
                    if np.shape(a) != (self.trials, n):
                        raise ValueError("init_spins needs one [trials, n_k] array per instance")
                init = np.ascontiguousarray(np.concatenate([_spins_int8(a).reshape(-1) for a in parts]))
        self._handle = ctypes.c_void_p()
        self.stream = stream if stream is not None else current_stream()
        _check(lib.pim_batch_create(arr, self.count, self.trials, _ptr(init, ctypes.c_int8), self.stream,
                                    ctypes.byref(self._handle)))

    def run(self, beta, eta, seed, start_step=0, kernel="mfma", target=None, stream=None, record=False):
        """One pim_run: kernel "mfma" (int8 / FP8 / BF16 matrix cores), "f4"
        (as "mfma", but couplings in {0, +-1, +-2, +-3, +-4, +-6} run on e2m1
        operands, identical results), "plain" or "seq"."""
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        if beta.shape != eta.shape or beta.ndim != 1:
            raise ValueError("beta and eta must be 1-D arrays of equal length")
        sc = Schedule()
        sc.steps = beta.size
        sc.beta = _ptr(beta, ctypes.c_double)
        sc.eta = _ptr(eta, ctypes.c_double)
        sc.start_step = int(start_step)
        sc.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        sc.record_states = 1 if record else 0
        self._steps = beta.size
        tgt = None
        if target is not None:
            tgt = np.ascontiguousarray(np.broadcast_to(np.asarray(target, dtype=np.float64), (self.count,)))
            sc.use_target = 1
            sc.target = _ptr(tgt, ctypes.c_double)
        if stream is not None:
            self.stream = stream
        _check(lib.pim_run(self._handle, ctypes.byref(sc), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                           self.stream))
        self._keep = (beta, eta, tgt)
        return self

    def cancel(self):
        _check(lib.pim_cancel(self._handle))

    def tune(self, steps=200):
        """Autotunes waves per workgroup for every distinct N (see pim_tune)."""
        out = np.zeros(len(set(self.ns)), np.int32)
        _check(lib.pim_tune(self._handle, int(steps), self.stream, _ptr(out, ctypes.c_int32)))
        return out

    def best(self, k):
        """(spins int8[n], energy, trial, step) of the lowest-energy candidate."""
        spins = np.zeros(self.ns[k], dtype=np.int8)
        e = ctypes.c_double()
        tr = ctypes.c_int32()
        st = ctypes.c_int32()
        _check(lib.pim_best(self._handle, int(k), _ptr(spins, ctypes.c_int8), ctypes.byref(e),
                            ctypes.byref(tr), ctypes.byref(st)))
        return spins, e.value, tr.value, st.value

    def trials_of(self, k, spins=True):
        R, n = self.trials, self.ns[k]
        out = {
            "e_best": np.zeros(R, np.float64), "t_best": np.zeros(R, np.int32),
            "first_hit": np.zeros(R, np.int32), "e_final": np.zeros(R, np.float64),
        }
        bs = np.zeros((R, n), np.int8) if spins else None
        fs = np.zeros((R, n), np.int8) if spins else None
        _check(lib.pim_trials(self._handle, int(k), _ptr(out["e_best"], ctypes.c_double),
                              _ptr(out["t_best"], ctypes.c_int32), _ptr(out["first_hit"], ctypes.c_int32),
                              _ptr(out["e_final"], ctypes.c_double), _ptr(bs, ctypes.c_int8),
                              _ptr(fs, ctypes.c_int8)))
        if spins:
            out["best_state"] = bs
            out["final"] = fs
        return out

    def states(self, k, trial):
        """Recorded trajectory of one trial: int8 [T + 1, n] (run with record=True)."""
        out = np.zeros((self._steps + 1, self.ns[k]), np.int8)
        _check(lib.pim_states(self._handle, int(k), int(trial), _ptr(out, ctypes.c_int8)))
        return out

    def flip_counts(self, k):
        """(num, den) of the neighbour-triggered flip rate, int64 [T] each."""
        num = np.zeros(self._steps, np.int64)
        den = np.zeros(self._steps, np.int64)
        _check(lib.pim_flip_counts(self._handle, int(k), _ptr(num, ctypes.c_int64), _ptr(den, ctypes.c_int64)))
        return num, den

    def kernel_ms(self):
        ms = ctypes.c_float()
        _check(lib.pim_kernel_time(self._handle, ctypes.byref(ms)))
        return ms.value

    def close(self):
        if self._handle:
            lib.pim_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Server:
    """Request server with continuous batching (see pim_server_* in pim.h):
    submit real-valued Ising requests as they arrive, flush to launch what is
    staged, poll for finished requests."""

    def __init__(self, *, max_n, trials, beta, eta, j_scale=1.0, xi=2.0, levels=4, noise="gauss",
                 noise_table=None, prec="fp8", slots_per_class=4096, max_batch=256, streams=4, seed=1,
                 hbm_budget=0, poll_max=4096, max_wait_us=0.0, prealloc_chunks=0, mimo=False):
        _device_ready()
        self.mimo = bool(mimo)
        self._poll_max = max(int(poll_max), int(max_batch))
        self._ids = np.zeros(self._poll_max, np.uint32)
        self._states = np.zeros((self._poll_max, MAX_N_LDS), np.int8)
        self._e = np.zeros(self._poll_max, np.float64)
        self._t = np.zeros((self._poll_max, 3), np.float64)
        self._xm = np.zeros((self._poll_max, MAX_N_LDS // 2), np.float64)
        self._beta = np.ascontiguousarray(beta, dtype=np.float64)
        self._eta = np.ascontiguousarray(eta, dtype=np.float64)
        self._ztab = None if noise_table is None else np.ascontiguousarray(noise_table, dtype=np.float64)
        c = ServerConfig()
        c.max_n, c.slots_per_class, c.max_batch = int(max_n), int(slots_per_class), int(max_batch)
        c.trials, c.steps = int(trials), self._beta.size
        c.beta, c.eta = _ptr(self._beta, ctypes.c_double), _ptr(self._eta, ctypes.c_double)
        c.j_scale, c.xi, c.levels = float(j_scale), float(xi), int(levels)
        c.noise = _NOISES[noise] if isinstance(noise, str) else int(noise)
        c.noise_table = _ptr(self._ztab, ctypes.c_double)
        c.prec = _PRECS[prec]
        c.streams, c.seed, c.hbm_budget = int(streams), int(seed), int(hbm_budget)
        c.max_wait_us = float(max_wait_us)
        c.prealloc_chunks = int(prealloc_chunks)
        self._handle = ctypes.c_void_p()
        create = lib.pim_server_create_mimo if self.mimo else lib.pim_server_create
        _check(create(ctypes.byref(c), ctypes.byref(self._handle)))

    def submit(self, ids, Js, hs=None):
        """Stages requests (ids, J arrays, h arrays); returns how many were
        admitted.  A rejected request raises PimError whose `admitted` is the
        number of requests before it that were admitted."""
        k = len(ids)
        if k == 0:
            return 0
        Js = [np.ascontiguousarray(J, dtype=np.float64) for J in Js]
        hs = None if hs is None else [np.ascontiguousarray(h, dtype=np.float64) for h in hs]
        idarr = np.ascontiguousarray(ids, dtype=np.uint32)
        if len(Js) != k or idarr.shape != (k,) or (hs is not None and len(hs) != k):
            raise ValueError("ids, Js and hs must have one entry per request")
        for J in Js:
            if J.ndim != 2 or J.shape[0] != J.shape[1]:
                raise ValueError("each J must be a square matrix")
        if hs is not None:
            for J, h in zip(Js, hs):
                if h.shape != (J.shape[0],):
                    raise ValueError("each h must have one entry per spin")
        # the library reads the arrays through these addresses during the call
        ns = np.fromiter((J.shape[0] for J in Js), dtype=np.int32, count=k)
        jp = np.fromiter((J.ctypes.data for J in Js), dtype=np.uintp, count=k)
        hp = None if hs is None else np.fromiter((h.ctypes.data for h in hs), dtype=np.uintp, count=k)
        adm = ctypes.c_int32()
        st = lib.pim_server_submit(self._handle, k, idarr.ctypes.data, ns.ctypes.data, jp.ctypes.data,
                                   None if hp is None else hp.ctypes.data, ctypes.byref(adm))
        if st != PIM_OK:
            # the requests before the rejected one are admitted; the error says how many
            err = PimError(st, lib.pim_last_error().decode(errors="replace"))
            err.admitted = adm.value
            raise err
        return adm.value

    def submit_mimo(self, ids, Hs, ys, qams, mappings="di", esn0s=1.0):
        """Stages MIMO requests (server created with mimo=True): complex H
        [nr, nt] and y [nr] per request, its modulation, mapping and Es/N0;
        returns how many were admitted."""
        k = len(ids)
        if k == 0:
            return 0
        Hc = [_complex_interleaved(H) for H in Hs]
        yc = [_complex_interleaved(y) for y in ys]
        qams = np.broadcast_to(np.asarray(qams), (k,))
        maps = np.broadcast_to(np.asarray(mappings), (k,))
        dims = np.zeros((k, 4), np.int32)
        for r in range(k):
            if Hc[r].ndim != 3 or yc[r].shape != (Hc[r].shape[0], 2):
                raise ValueError("each H must be [nr, nt] and y [nr]")
            dims[r] = (Hc[r].shape[0], Hc[r].shape[1], int(qams[r]), _MAPS[str(maps[r])])
        esn0 = np.ascontiguousarray(np.broadcast_to(np.asarray(esn0s, np.float64), (k,)))
        hp = np.fromiter((a.ctypes.data for a in Hc), dtype=np.uintp, count=k)
        yp = np.fromiter((a.ctypes.data for a in yc), dtype=np.uintp, count=k)
        return self.submit_mimo_raw(np.asarray(ids, np.uint32), dims, esn0, hp, yp)

    def submit_mimo_raw(self, ids, dims, esn0, hptrs, yptrs):
        """submit_mimo on prepared arrays: ids uint32 [k], dims int32 [k, 4]
        (nr, nt, qam, mapping code), esn0 float64 [k], and the addresses of
        each request's interleaved H and y (uintp [k]), which must stay valid
        during the call."""
        k = len(ids)
        if k == 0:
            return 0
        ids = np.ascontiguousarray(ids, np.uint32)
        dims = np.ascontiguousarray(dims, np.int32)
        esn0 = np.ascontiguousarray(esn0, np.float64)
        hptrs = np.ascontiguousarray(hptrs, np.uintp)
        yptrs = np.ascontiguousarray(yptrs, np.uintp)
        if dims.shape != (k, 4) or esn0.shape != (k,) or hptrs.shape != (k,) or yptrs.shape != (k,):
            raise ValueError("ids, dims, esn0 and the pointer arrays must have one entry per request")
        adm = ctypes.c_int32()
        st = lib.pim_server_submit_mimo(self._handle, k, ids.ctypes.data, dims.ctypes.data, esn0.ctypes.data,
                                        hptrs.ctypes.data, yptrs.ctypes.data, ctypes.byref(adm))
        if st != PIM_OK:
            err = PimError(st, lib.pim_last_error().decode(errors="replace"))
            err.admitted = adm.value
            raise err
        return adm.value

    def poll_mimo(self, states=True):
        """poll_times() plus x_m [k, MAX_N_LDS // 2] per request (first 2 nt
        entries used)."""
        done = ctypes.c_int32()
        _check(lib.pim_server_poll_mimo(self._handle, self._poll_max, _ptr(self._ids, ctypes.c_uint32),
                                        _ptr(self._states, ctypes.c_int8) if states else None,
                                        _ptr(self._e, ctypes.c_double), _ptr(self._xm, ctypes.c_double),
                                        _ptr(self._t, ctypes.c_double), ctypes.byref(done)))
        k = done.value
        return (self._ids[:k].copy(), (self._states[:k].copy() if states else None), self._e[:k].copy(),
                self._xm[:k].copy(), self._t[:k].copy())

    def flush(self):
        n = ctypes.c_int32()
        _check(lib.pim_server_flush(self._handle, ctypes.byref(n)))
        return n.value

    def poll(self, states=True):
        """Finished requests (copies): (ids uint32 [k], states int8 [k, MAX_N_LDS]
        or None, energies [k]); at most `poll_max` per call."""
        done = ctypes.c_int32()
        _check(lib.pim_server_poll(self._handle, self._poll_max, _ptr(self._ids, ctypes.c_uint32),
                                   _ptr(self._states, ctypes.c_int8) if states else None,
                                   _ptr(self._e, ctypes.c_double), ctypes.byref(done)))
        k = done.value
        return self._ids[:k].copy(), (self._states[:k].copy() if states else None), self._e[:k].copy()

    def poll_times(self, states=True):
        """poll() plus, per request, (admitted, launched, seen finished) in
        seconds of the host's monotonic clock (time.perf_counter's clock)."""
        done = ctypes.c_int32()
        _check(lib.pim_server_poll_times(self._handle, self._poll_max, _ptr(self._ids, ctypes.c_uint32),
                                         _ptr(self._states, ctypes.c_int8) if states else None,
                                         _ptr(self._e, ctypes.c_double), _ptr(self._t, ctypes.c_double),
                                         ctypes.byref(done)))
        k = done.value
        return (self._ids[:k].copy(), (self._states[:k].copy() if states else None), self._e[:k].copy(),
                self._t[:k].copy())

    def pending(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.pim_server_pending(self._handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self._handle:
            lib.pim_server_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
