"""Python binding of libafqmc (ctypes).  Argument marshalling only: every step
of the walker propagation runs in the library's HIP kernels; PyTorch only
supplies the HIP stream and, optionally, device memory for explicit fields.

The library must have been built (``python -m paper_1703_01545_amd.build``);
importing this module without it raises ImportError — there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# AFQMC_LIB may name another build of the same sources (e.g. for A/B timing)
LIB_PATH = os.environ.get("AFQMC_LIB") or os.path.join(_HERE, "libafqmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libafqmc.so not built at {LIB_PATH}; run python -m paper_1703_01545_amd.build")

_lib = C.CDLL(LIB_PATH)

OK, E_INVALID, E_SHAPE, E_NOMEM, E_DEVICE, E_SINGULAR, E_STATE = 0, -1, -2, -3, -4, -5, -6
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16_plain": 3, "bf16x3": 4}
MODE = {"phaseless": 0, "free": 1}

# Every C-ABI entry point declared in include/afqmc.h.
EXPORTS = [
    "afqmc_load_hamiltonian", "afqmc_init_walkers", "afqmc_step", "afqmc_local_energy",
    "afqmc_orthonormalize", "afqmc_pair_step", "afqmc_pair_batch_step", "afqmc_get_walkers",
    "afqmc_sys_info", "afqmc_checkpoint", "afqmc_restore", "afqmc_free_sys", "afqmc_free_ham",
    "afqmc_last_error", "afqmc_selftest_gemm", "afqmc_selftest_gemm_shape", "afqmc_selftest_fields", "afqmc_profile_enable",
    "afqmc_profile_read", "afqmc_phase_name", "afqmc_selftest_propagate", "afqmc_autotune",
    "afqmc_adjoint_forward", "afqmc_adjoint_backward", "afqmc_pair_step_noalloc",
    "afqmc_population_control", "afqmc_init_from_primary", "afqmc_cap_events",
    "afqmc_init_walkers_msd", "afqmc_gs_monitor", "afqmc_tune_cache_save",
    "afqmc_tune_cache_load", "afqmc_tune_cache_clear",
]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("taylor_order", C.c_int), ("ortho_every", C.c_int),
                ("measure_every", C.c_int), ("contract_prec", C.c_int), ("mode", C.c_int),
                ("fb_cap", C.c_double), ("caps_enabled", C.c_int)]


_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_lib.afqmc_last_error.restype = C.c_char_p
_lib.afqmc_load_hamiltonian.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, _vp, C.POINTER(_vp)]
_lib.afqmc_init_walkers.argtypes = [_vp, C.c_int, C.c_int, _dp, _dp, C.c_int, C.POINTER(Params),
                                    C.POINTER(_vp)]
_lib.afqmc_init_walkers_msd.argtypes = [_vp, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_int,
                                        C.POINTER(Params), C.POINTER(_vp)]
_lib.afqmc_step.argtypes = [_vp, C.c_uint64, C.c_uint64, C.c_int, _vp]
_lib.afqmc_local_energy.argtypes = [_vp, _dp, _dp, _dp]
_lib.afqmc_orthonormalize.argtypes = [_vp]
_lib.afqmc_population_control.argtypes = [_vp, C.c_double]
_lib.afqmc_cap_events.argtypes = [_vp, C.POINTER(C.c_int64)]
_lib.afqmc_init_from_primary.argtypes = [_vp, _vp]
_lib.afqmc_pair_step.argtypes = [_vp, _vp, C.c_uint64, C.c_int, _vp, _dp]
_lib.afqmc_pair_step_noalloc.argtypes = [_vp, _vp, C.c_uint64, C.c_int, _vp, _dp]
_lib.afqmc_pair_batch_step.argtypes = [C.c_int, C.POINTER(_vp), C.POINTER(_vp),
                                       C.POINTER(C.c_uint64), C.c_int, C.c_int, C.c_int, _dp]
_lib.afqmc_autotune.argtypes = [_vp, C.POINTER(C.c_int)]
_lib.afqmc_adjoint_forward.argtypes = [_vp, _dp, C.c_uint64, C.c_int, C.c_int, C.c_int, _dp]
_lib.afqmc_adjoint_backward.argtypes = [_vp, _dp]
_lib.afqmc_get_walkers.argtypes = [_vp, _dp, _dp, _dp, C.POINTER(C.c_ubyte)]
_lib.afqmc_sys_info.argtypes = [_vp] + [C.POINTER(C.c_int)] * 5 + [C.POINTER(C.c_int64)]
_lib.afqmc_checkpoint.argtypes = [_vp, _vp, C.POINTER(C.c_size_t)]
_lib.afqmc_restore.argtypes = [_vp, _vp, C.c_size_t]
_lib.afqmc_free_sys.argtypes = [_vp]
_lib.afqmc_free_sys.restype = None
_lib.afqmc_free_ham.argtypes = [_vp]
_lib.afqmc_free_ham.restype = None
_lib.afqmc_selftest_gemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
_lib.afqmc_tune_cache_save.argtypes = [C.c_char_p]
_lib.afqmc_tune_cache_load.argtypes = [C.c_char_p]
_lib.afqmc_tune_cache_clear.argtypes = []
_lib.afqmc_gs_monitor.argtypes = [_vp, C.c_double, _dp, _dp, C.POINTER(C.c_int64)]
_lib.afqmc_selftest_gemm_shape.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                             _dp, _dp, _dp]
_lib.afqmc_selftest_fields.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int, C.c_int, _dp]
_lib.afqmc_selftest_propagate.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                           _dp, _dp, _dp, _dp]
_lib.afqmc_profile_enable.argtypes = [_vp, C.c_int]
_lib.afqmc_profile_read.argtypes = [_vp, C.c_int, _dp, C.POINTER(C.c_int64)]
_lib.afqmc_phase_name.argtypes = [C.c_int]
_lib.afqmc_phase_name.restype = C.c_char_p
for _n in EXPORTS:
    if _n not in ("afqmc_last_error", "afqmc_free_sys", "afqmc_free_ham", "afqmc_phase_name"):
        getattr(_lib, _n).restype = C.c_int


class AfqmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"afqmc status {status}: {msg}")
        self.status = status


def _check(status: int):
    if status != OK:
        raise AfqmcError(status, _lib.afqmc_last_error().decode(errors="replace"))


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _current_stream() -> int:
    import torch
    if not torch.cuda.is_available():
        return 0
    return int(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(fields) -> Optional[int]:
    """Device pointer of an explicit-field tensor (torch, float64, on the GPU)."""
    if fields is None:
        return None
    import torch
    if not (isinstance(fields, torch.Tensor) and fields.is_cuda and fields.dtype == torch.float64
            and fields.is_contiguous()):
        raise TypeError("fields must be a contiguous float64 torch tensor on the GPU")
    return int(fields.data_ptr())


class Hamiltonian:
    """h (M x M), chol (n_chol x M x M) and e_core of Eq. 1, resident on the GPU."""

    def __init__(self, h, chol, e_core: float = 0.0, stream: Optional[int] = None):
        h = _f64(h)
        chol = _f64(chol)
        self.M = h.shape[0]
        self.n_chol = chol.shape[0]
        assert h.shape == (self.M, self.M) and chol.shape[1:] == (self.M, self.M)
        self.stream = _current_stream() if stream is None else int(stream)
        out = _vp()
        _check(_lib.afqmc_load_hamiltonian(self.M, self.n_chol, _ptr(h), _ptr(chol), float(e_core),
                                           _vp(self.stream), C.byref(out)))
        self._h = out

    def free(self):
        if self._h:
            _lib.afqmc_free_ham(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class System:
    """One system (trial + walker batch) on a Hamiltonian."""

    def __init__(self, ham: Hamiltonian, n_alpha: int, n_beta: int, trial, n_walkers: int,
                 dt: float, taylor_order: int = 6, ortho_every: int = 10, measure_every: int = 20,
                 precision: str = "fp64", mode: str = "phaseless", init_phi=None,
                 fb_cap: float = 0.0, caps_enabled: bool = False, expansion=None):
        """expansion: optional (coefficients (n_det,), determinants (n_det, M, N))
        of a multi-determinant trial; `trial` is then ignored."""
        self.ham = ham
        self.M, self.n_chol = ham.M, ham.n_chol
        self.na, self.nb = int(n_alpha), int(n_beta)
        self.N = self.na + self.nb
        self.nw = int(n_walkers)
        self.mode = mode
        trial = _f64(trial if expansion is None else expansion[1][0])
        assert trial.shape == (self.M, self.N)
        init = None if init_phi is None else _f64(init_phi)
        self.params = Params(float(dt), int(taylor_order), int(ortho_every), int(measure_every),
                             PREC[precision], MODE[mode], float(fb_cap), int(bool(caps_enabled)))
        out = _vp()
        if expansion is None:
            _check(_lib.afqmc_init_walkers(ham._h, self.na, self.nb, _ptr(trial), _ptr(init),
                                           self.nw, C.byref(self.params), C.byref(out)))
        else:
            coeffs, dets = _f64(expansion[0]), _f64(expansion[1])
            assert dets.shape == (len(coeffs), self.M, self.N)
            _check(_lib.afqmc_init_walkers_msd(ham._h, self.na, self.nb, len(coeffs), _ptr(coeffs),
                                               _ptr(dets), _ptr(init), self.nw,
                                               C.byref(self.params), C.byref(out)))
        self._s = out

    def step(self, n_steps: int = 1, seed: int = 0, stream_id: int = 0, fields=None):
        _check(_lib.afqmc_step(self._s, int(seed), int(stream_id), int(n_steps),
                               _dev_ptr(fields)))

    def orthonormalize(self):
        _check(_lib.afqmc_orthonormalize(self._s))

    def cap_events(self) -> int:
        """(live walker, step, gamma) events with |xbar| above fb_cap so far."""
        n = C.c_int64()
        _check(_lib.afqmc_cap_events(self._s, C.byref(n)))
        return n.value

    def gs_monitor(self, threshold: float = 9.0):
        """Gram-Schmidt monitor since the last call: (largest loss of
        orthogonality ell, largest |ln |det R||, spin blocks with ell above
        threshold); clears the record."""
        me, ml, n = C.c_double(), C.c_double(), C.c_int64()
        _check(_lib.afqmc_gs_monitor(self._s, float(threshold), C.byref(me), C.byref(ml),
                                     C.byref(n)))
        return me.value, ml.value, n.value

    def population_control(self, xi: float):
        """Comb of the walker population with the uniform number xi in [0, 1)."""
        _check(_lib.afqmc_population_control(self._s, float(xi)))

    def init_from_primary(self, primary: "System"):
        """Start this (secondary) system from the primary's walkers (PES)."""
        _check(_lib.afqmc_init_from_primary(self._s, primary._s))

    def local_energy(self):
        el = np.empty((self.nw, 2))
        w = np.empty((self.nw, 2) if self.mode == "free" else self.nw)
        em = np.empty(1)
        _check(_lib.afqmc_local_energy(self._s, _ptr(el), _ptr(w), _ptr(em)))
        wv = w[:, 0] + 1j * w[:, 1] if self.mode == "free" else w
        return el[:, 0] + 1j * el[:, 1], wv, float(em[0])

    def walkers(self):
        phi = np.empty((self.nw, 2, self.N, self.M))
        w = np.empty((self.nw, 2) if self.mode == "free" else self.nw)
        lo = np.empty((self.nw, 2))
        alive = np.empty(self.nw, dtype=np.uint8)
        _check(_lib.afqmc_get_walkers(self._s, _ptr(phi), _ptr(w), _ptr(lo),
                                      alive.ctypes.data_as(C.POINTER(C.c_ubyte))))
        phic = np.swapaxes(phi[:, 0] + 1j * phi[:, 1], 1, 2)   # (nw, M, N)
        wv = w[:, 0] + 1j * w[:, 1] if self.mode == "free" else w
        return dict(phi=phic, weight=wv, lnov=lo[:, 0] + 1j * lo[:, 1], alive=alive.astype(bool))

    def info(self):
        v = [C.c_int() for _ in range(5)]
        t = C.c_int64()
        _check(_lib.afqmc_sys_info(self._s, *[C.byref(x) for x in v], C.byref(t)))
        return dict(M=v[0].value, n_chol=v[1].value, n_alpha=v[2].value, n_beta=v[3].value,
                    n_walkers=v[4].value, step=t.value)

    def profile(self, enable: bool = True):
        """Start (clearing the counters) or stop per-phase HIP-event timing."""
        _check(_lib.afqmc_profile_enable(self._s, 1 if enable else 0))

    def profile_read(self):
        """{phase name: (total ms, launches)} since profiling was enabled."""
        out = {}
        i = 0
        while True:
            name = _lib.afqmc_phase_name(i)
            if name is None:
                break
            ms = C.c_double()
            n = C.c_int64()
            _check(_lib.afqmc_profile_read(self._s, i, C.byref(ms), C.byref(n)))
            out[name.decode()] = (ms.value, n.value)
            i += 1
        return out

    def adjoint_forward(self, V, n_steps: int, seed: int = 0, checkpoint_every: int = 10,
                        precision: str = "fp64") -> float:
        """Advance n_steps (device fields) keeping snapshots; returns the mixed
        energy at the end.  See afqmc_adjoint_backward for dE/dlambda."""
        V = _f64(V)
        assert V.shape == (self.M, self.M)
        e = C.c_double()
        _check(_lib.afqmc_adjoint_forward(self._s, _ptr(V), int(seed), int(n_steps),
                                          int(checkpoint_every), PREC[precision], C.byref(e)))
        return e.value

    def adjoint_backward(self) -> float:
        """dE/dlambda of the last adjoint_forward window for h -> h + lambda V."""
        d = C.c_double()
        _check(_lib.afqmc_adjoint_backward(self._s, C.byref(d)))
        return d.value

    def checkpoint(self) -> bytes:
        n = C.c_size_t()
        _check(_lib.afqmc_checkpoint(self._s, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(_lib.afqmc_checkpoint(self._s, C.cast(buf, _vp), C.byref(n)))
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(_lib.afqmc_restore(self._s, C.cast(buf, _vp), len(blob)))

    def free(self):
        if getattr(self, "_s", None):
            _lib.afqmc_free_sys(self._s)
            self._s = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def tune_cache_save(path: str):
    """Write the launch shapes tuned in this process (tagged with the device)."""
    _check(_lib.afqmc_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str):
    """Add the launch shapes of a cache written on a device like this one;
    shapes tuned in this process keep their choice."""
    _check(_lib.afqmc_tune_cache_load(os.fsencode(path)))


def tune_cache_clear():
    """Empty the table of tuned launch shapes (systems keep their choices)."""
    _check(_lib.afqmc_tune_cache_clear())


def pair_step(a: System, b: System, n_steps: int, seed: int = 0, fields=None) -> np.ndarray:
    """Correlated pair (Sec. II.B); returns the (n_meas, 3) trace E_a, E_b, dE."""
    me = a.params.measure_every
    t0 = a.info()["step"]
    n_meas = sum(1 for i in range(n_steps) if me > 0 and (t0 + i + 1) % me == 0)
    tr = np.zeros((max(n_meas, 1), 3))
    _check(_lib.afqmc_pair_step(a._s, b._s, int(seed), int(n_steps), _dev_ptr(fields), _ptr(tr)))
    return tr[:n_meas]


def pair_step_noalloc(a: System, b: System, n_steps: int, seed: int = 0,
                      fields=None) -> np.ndarray:
    """pair_step through the entry point that allocates no device memory
    during the call (its trace staging is a fixed array in the library, at
    most NOALLOC_MAX_MEASUREMENTS measurements per call)."""
    me = a.params.measure_every
    t0 = a.info()["step"]
    n_meas = sum(1 for i in range(n_steps) if me > 0 and (t0 + i + 1) % me == 0)
    tr = np.zeros((max(n_meas, 1), 3))
    _check(_lib.afqmc_pair_step_noalloc(a._s, b._s, int(seed), int(n_steps), _dev_ptr(fields),
                                        _ptr(tr)))
    return tr[:n_meas]


NOALLOC_MAX_MEASUREMENTS = 1024


def pair_batch_step(pairs, seeds, n_steps: int, lanes: int = 0, graph: bool = True) -> np.ndarray:
    """Many pairs advanced together (graph-replayed unless graph=False);
    returns (n_pairs, n_meas, 3)."""
    n = len(pairs)
    me = pairs[0][0].params.measure_every
    t0 = pairs[0][0].info()["step"]
    n_meas = sum(1 for i in range(n_steps) if me > 0 and (t0 + i + 1) % me == 0)
    A = (_vp * n)(*[p[0]._s for p in pairs])
    B = (_vp * n)(*[p[1]._s for p in pairs])
    S = (C.c_uint64 * n)(*[int(s) for s in seeds])
    tr = np.zeros((n, max(n_meas, 1), 3))
    _check(_lib.afqmc_pair_batch_step(n, A, B, S, int(n_steps), int(lanes), 0 if graph else 1,
                                      _ptr(tr)))
    return tr[:, :n_meas]


def autotune(system: System):
    """Autotune the system's launch shapes; returns (force-bias tile,
    field-sum tile, propagation shape)."""
    ch = (C.c_int * 3)()
    _check(_lib.afqmc_autotune(system._s, ch))
    return tuple(ch)


def selftest_gemm(A, B, precision: str = "fp64") -> np.ndarray:
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    n = B.shape[0]
    Cm = np.empty((m, n))
    _check(_lib.afqmc_selftest_gemm(PREC[precision], m, n, k, _ptr(A), _ptr(B), _ptr(Cm)))
    return Cm


def selftest_gemm_shape(A, B, precision: str, tile: int, ksplit: int = 1) -> np.ndarray:
    """C = A B^T with the workgroup tile (0 heuristic, 1 64x64, 2 128x128,
    3 256x128, 4 256x128 over 16 wavefronts) and the number of K ranges fixed; FP32 operand storage for
    fp32 and bf16 (split-BF16 products)."""
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    n = B.shape[0]
    Cm = np.empty((m, n))
    _check(_lib.afqmc_selftest_gemm_shape(PREC[precision], tile, ksplit, m, n, k, _ptr(A), _ptr(B),
                                          _ptr(Cm)))
    return Cm


def selftest_propagate(phi, P, A, K: int, precision: str = "fp64", variant: int = 0) -> np.ndarray:
    """phi: (nw, M, N) complex, P: (M, M) real, A: (nw, M, M) complex symmetric ->
    P T_K(A) P phi computed by the fused propagation kernel."""
    phi = np.asarray(phi)
    nw, M, N = phi.shape
    ph = _f64(np.stack([np.swapaxes(phi.real, 1, 2), np.swapaxes(phi.imag, 1, 2)], axis=1))
    Ah = _f64(np.stack([A.real, A.imag], axis=1))
    out = np.empty_like(ph)
    _check(_lib.afqmc_selftest_propagate(PREC[precision], M, N, nw, int(K), int(variant), _ptr(ph),
                                         _ptr(_f64(P)), _ptr(Ah), _ptr(out)))
    return np.swapaxes(out[:, 0] + 1j * out[:, 1], 1, 2)


def selftest_fields(seed: int, stream_id: int, t: int, nw: int, n_chol: int) -> np.ndarray:
    out = np.empty((nw, n_chol))
    _check(_lib.afqmc_selftest_fields(int(seed), int(stream_id), int(t), nw, n_chol, _ptr(out)))
    return out
