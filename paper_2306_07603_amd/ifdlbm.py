"""Python binding of libifdlbm.so: the C ABI of include/ifdlbm.h, call by call.

Only argument marshalling happens here (numpy host arrays and torch device
tensors in, ctypes pointers out); every step of the method runs in the HIP
kernels of the library.  Loading fails loudly when the library is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

try:   # load torch's HIP runtime first so that torch and the library share one
    import torch  # noqa: F401
except ImportError:
    torch = None

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libifdlbm.so")

IFDLBM_OK = 0
IFDLBM_EINVAL = -1
IFDLBM_ENOMEM = -2
IFDLBM_EDEVICE = -3
IFDLBM_EDIVERGED = -4
IFDLBM_ENOTCONVERGED = -5

IFDLBM_FP64, IFDLBM_FP32, IFDLBM_FP16DEV, IFDLBM_FP32X, IFDLBM_FP32SR, IFDLBM_FP32SRF = 0, 1, 2, 3, 4, 5
IFDLBM_KERNEL_FUSED, IFDLBM_KERNEL_STAGED = 0, 1
IFDLBM_DT_CONTRAVARIANT, IFDLBM_DT_CARTESIAN = 0, 1
IFDLBM_STATUS_RUNNING, IFDLBM_STATUS_CONVERGED, IFDLBM_STATUS_DIVERGED, IFDLBM_STATUS_NOT_CONVERGED = 0, 1, 2, 3

PRECISIONS = {"fp64": IFDLBM_FP64, "fp32": IFDLBM_FP32, "fp16dev": IFDLBM_FP16DEV, "fp32x": IFDLBM_FP32X, "fp32sr": IFDLBM_FP32SR,
              "fp32srf": IFDLBM_FP32SRF}
KERNELS = {"fused": IFDLBM_KERNEL_FUSED, "staged": IFDLBM_KERNEL_STAGED}


class IfdlbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (code %d): %s" % (_strerror(code), code, message))
        self.code = code


class ifdlbm_cavity(ctypes.Structure):
    _fields_ = [("n_xi", ctypes.c_int32), ("n_eta", ctypes.c_int32), ("re", ctypes.c_double),
                ("n", ctypes.c_double), ("theta_deg", ctypes.c_double), ("u_lid", ctypes.c_double)]


class ifdlbm_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cfl", ctypes.c_double), ("mix", ctypes.c_double),
                ("rho0", ctypes.c_double), ("gamma_min", ctypes.c_double), ("residual_every", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("batched", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("dt_rule", ctypes.c_int32), ("segment_rows", ctypes.c_int32), ("lambda_mode", ctypes.c_int32),
                ("pressure_residual", ctypes.c_int32), ("hip_stream", ctypes.c_void_p)]


class ifdlbm_info_t(ctypes.Structure):
    _fields_ = [("n_cavities", ctypes.c_int32), ("n_active", ctypes.c_int32), ("nodes", ctypes.c_int64),
                ("state_bytes", ctypes.c_int64), ("alg_bytes_per_node", ctypes.c_double),
                ("launches_per_step", ctypes.c_int32), ("work_items", ctypes.c_int64)]


class ifdlbm_regime_t(ctypes.Structure):
    _fields_ = [("regime", ctypes.c_int32), ("mean", ctypes.c_double), ("rel_amplitude", ctypes.c_double),
                ("f_main", ctypes.c_double), ("f_second", ctypes.c_double), ("harmonic_fraction", ctypes.c_double),
                ("second_fraction", ctypes.c_double)]


IFDLBM_LAMBDA_LAGGED = 0
IFDLBM_LAMBDA_IMPLICIT = 1
IFDLBM_EP_MEAN_REMOVED = 0
IFDLBM_EP_PRINTED = 1

IFDLBM_REGIME_STEADY = 0
IFDLBM_REGIME_PERIODIC = 1
IFDLBM_REGIME_QUASI_PERIODIC = 2
IFDLBM_REGIME_APERIODIC = 3
REGIMES = {0: "steady", 1: "periodic", 2: "quasi-periodic", 3: "aperiodic"}

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p


def lib():
    """The loaded libifdlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libifdlbm.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        verify_build(L)
        L.ifdlbm_default_options.argtypes = [ctypes.POINTER(ifdlbm_options)]
        L.ifdlbm_create.argtypes = [ctypes.POINTER(ifdlbm_cavity), ctypes.c_int32, ctypes.POINTER(ifdlbm_options),
                                    ctypes.POINTER(_H)]
        L.ifdlbm_step.argtypes = [_H, ctypes.c_int64]
        L.ifdlbm_sync.argtypes = [_H]
        L.ifdlbm_run_to_steady.argtypes = [_H, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _D, _D]
        L.ifdlbm_get_residuals.argtypes = [_H, _D, _D]
        L.ifdlbm_get_pressure_residuals.argtypes = [_H, _D, _D]
        L.ifdlbm_get_fields.argtypes = [_H, ctypes.c_int32, _D, _D, _D]
        L.ifdlbm_get_fields_device.argtypes = [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int32]
        L.ifdlbm_round_stochastic_device.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                     ctypes.c_void_p]
        L.ifdlbm_power_law_device.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_void_p]
        L.ifdlbm_kinetic_energy.argtypes = [_H, ctypes.c_int32, _D]
        L.ifdlbm_get_state.argtypes = [_H, ctypes.c_int32, _D, _D]
        L.ifdlbm_set_state.argtypes = [_H, ctypes.c_int32, _D, _D]
        L.ifdlbm_status.argtypes = [_H, ctypes.c_int32]
        L.ifdlbm_info.argtypes = [_H, ctypes.POINTER(ifdlbm_info_t)]
        L.ifdlbm_gradient.argtypes = [ctypes.POINTER(ifdlbm_cavity), ctypes.POINTER(ifdlbm_options), ctypes.c_int64,
                                      ctypes.c_int32, _D, _D]
        L.ifdlbm_gradient_noalloc.argtypes = [ctypes.POINTER(ifdlbm_cavity), ctypes.POINTER(ifdlbm_options),
                                              ctypes.c_int64, ctypes.c_int32, _D, _D]
        L.ifdlbm_adjoint.argtypes = [ctypes.POINTER(ifdlbm_cavity), ctypes.POINTER(ifdlbm_options), ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32, _D, _D]
        L.ifdlbm_autotune.argtypes = [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _D]
        L.ifdlbm_record.argtypes = [_H, ctypes.c_int32, ctypes.c_int32]
        L.ifdlbm_get_record.argtypes = [_H, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64), _D, _D, _D]
        L.ifdlbm_time_step.argtypes = [_H, ctypes.c_int32, _D]
        L.ifdlbm_classify.argtypes = [_D, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ifdlbm_regime_t)]
        L.ifdlbm_destroy.argtypes = [_H]
        L.ifdlbm_destroy.restype = None
        L.ifdlbm_strerror.argtypes = [ctypes.c_int]
        L.ifdlbm_strerror.restype = ctypes.c_char_p
        L.ifdlbm_last_error.argtypes = []
        L.ifdlbm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def verify_build(L) -> None:
    """Refuse a library built from other sources than the ones beside it (a stale build)."""
    from . import _build
    L.ifdlbm_build_digest.argtypes = []
    L.ifdlbm_build_digest.restype = ctypes.c_char_p
    built, here = L.ifdlbm_build_digest().decode(), _build.source_digest()
    if built != here:
        raise ImportError("%s was built from other sources (digest %s...) than those in %s (digest %s...); "
                          "rebuild with __graft_entry__.build()" % (LIB_PATH, built[:12], _build.CSRC, here[:12]))


def _strerror(code: int) -> str:
    return lib().ifdlbm_strerror(code).decode()


def _check(rc: int, allow=()) -> int:
    if rc < 0 and rc not in allow:
        raise IfdlbmError(rc, lib().ifdlbm_last_error().decode())
    return rc


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


@dataclass
class Cavity:
    """One cavity: grid size, Re of Eq. (2.15.1), n of Eq. (1.4), top angle, lid speed."""
    n_xi: int
    n_eta: int
    re: float
    n: float
    theta_deg: float
    u_lid: float = 0.1

    def c(self) -> ifdlbm_cavity:
        return ifdlbm_cavity(self.n_xi, self.n_eta, self.re, self.n, self.theta_deg, self.u_lid)


def ifdlbm_default_options(**overrides) -> ifdlbm_options:
    o = ifdlbm_options()
    _check(lib().ifdlbm_default_options(ctypes.byref(o)))
    names = {f[0] for f in ifdlbm_options._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError("unknown option %r" % k)
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "kernel" and isinstance(v, str):
            v = KERNELS[v]
        setattr(o, k, v)
    return o


class Handle:
    """Owner of an ifdlbm_t*; the cavities it was created with are kept for array shapes."""

    def __init__(self, ptr: int, cavities: Sequence[Cavity], options: ifdlbm_options):
        self.ptr = ctypes.c_void_p(ptr)
        self.cavities = list(cavities)
        self.options = options

    def shape(self, cav: int):
        c = self.cavities[cav]
        return (c.n_eta, c.n_xi)

    def close(self):
        if self.ptr:
            lib().ifdlbm_destroy(self.ptr)
            self.ptr = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ifdlbm_create(cavities: Sequence[Cavity], options: Optional[ifdlbm_options] = None) -> Handle:
    options = options or ifdlbm_default_options()
    arr = (ifdlbm_cavity * len(cavities))(*[c.c() for c in cavities])
    out = _H()
    _check(lib().ifdlbm_create(arr, len(cavities), ctypes.byref(options), ctypes.byref(out)))
    return Handle(out.value, cavities, options)


def ifdlbm_step(h: Handle, n_steps: int) -> None:
    _check(lib().ifdlbm_step(h.ptr, int(n_steps)))


def ifdlbm_sync(h: Handle) -> None:
    _check(lib().ifdlbm_sync(h.ptr))


def ifdlbm_run_to_steady(h: Handle, tol: float, max_steps: int):
    """Returns (code, steps_done, res_u, res_p); code is OK, ENOTCONVERGED or EDIVERGED."""
    n = len(h.cavities)
    steps = (ctypes.c_int64 * n)()
    ru, rp = np.zeros(n), np.zeros(n)
    rc = _check(lib().ifdlbm_run_to_steady(h.ptr, float(tol), int(max_steps), steps, _dptr(ru), _dptr(rp)),
                allow=(IFDLBM_ENOTCONVERGED, IFDLBM_EDIVERGED))
    return rc, np.array(steps[:], dtype=np.int64), ru, rp


def ifdlbm_get_residuals(h: Handle):
    n = len(h.cavities)
    ru, rp = np.zeros(n), np.zeros(n)
    _check(lib().ifdlbm_get_residuals(h.ptr, _dptr(ru), _dptr(rp)))
    return ru, rp


def ifdlbm_get_pressure_residuals(h: Handle):
    """(E(P) as printed, E(P) with the spatial mean of P removed) of Eq. (2.19), per cavity."""
    n = len(h.cavities)
    printed, mean_removed = np.zeros(n), np.zeros(n)
    _check(lib().ifdlbm_get_pressure_residuals(h.ptr, _dptr(printed), _dptr(mean_removed)))
    return printed, mean_removed


def ifdlbm_get_fields(h: Handle, cav: int):
    shp = h.shape(cav)
    u, v, p = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    _check(lib().ifdlbm_get_fields(h.ptr, cav, _dptr(u), _dptr(v), _dptr(p)))
    return u, v, p


def ifdlbm_get_fields_device(h: Handle, cav: int, u, v, p) -> None:
    """u, v, p: contiguous torch tensors of n_eta * n_xi float64 or float32 on the device.  With a caller
    stream in the options the copy is enqueued there; with the handle's own stream the call waits for it."""
    dt = {8: 0, 4: 1}[u.element_size()]
    for t in (u, v, p):
        assert t.is_contiguous() and t.numel() == h.shape(cav)[0] * h.shape(cav)[1] and t.element_size() == u.element_size()
    _check(lib().ifdlbm_get_fields_device(h.ptr, cav, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(p.data_ptr()), dt))


def ifdlbm_round_stochastic_device(v, r16, out, stream=None) -> None:
    """The storage modes' stochastic rounding of FP64 to FP32 on device tensors: v float64, r16 int32 (its low 16
    bits are the random number), out float32, all contiguous with the same number of elements; runs on `stream`
    (a torch stream, default the current one) and returns when out is written."""
    import torch
    assert v.dtype == torch.float64 and r16.dtype == torch.int32 and out.dtype == torch.float32
    assert v.is_contiguous() and r16.is_contiguous() and out.is_contiguous()
    assert v.numel() == r16.numel() == out.numel() and v.is_cuda and r16.is_cuda and out.is_cuda
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().ifdlbm_round_stochastic_device(ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(r16.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()), v.numel(), ctypes.c_void_p(s)))


def ifdlbm_power_law_device(x, y: float, out, stream=None) -> None:
    """The FP64 step's power x^y of Step (2) on device tensors: x and out float64, contiguous, with the same
    number of elements; runs on `stream` (a torch stream, default the current one) and returns when out is
    written."""
    import torch
    assert x.dtype == torch.float64 and out.dtype == torch.float64
    assert x.is_contiguous() and out.is_contiguous() and x.numel() == out.numel() and x.is_cuda and out.is_cuda
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().ifdlbm_power_law_device(ctypes.c_void_p(x.data_ptr()), float(y), ctypes.c_void_p(out.data_ptr()),
                                         x.numel(), ctypes.c_void_p(s)))


def ifdlbm_kinetic_energy(h: Handle, cav: int) -> float:
    e = ctypes.c_double()
    _check(lib().ifdlbm_kinetic_energy(h.ptr, cav, ctypes.byref(e)))
    return e.value


def ifdlbm_get_state(h: Handle, cav: int):
    ny, nx = h.shape(cav)
    F, L = np.zeros((9, ny, nx)), np.zeros((ny, nx))
    _check(lib().ifdlbm_get_state(h.ptr, cav, _dptr(F), _dptr(L)))
    return F, L


def ifdlbm_set_state(h: Handle, cav: int, F: np.ndarray, L: np.ndarray) -> None:
    ny, nx = h.shape(cav)
    F = np.ascontiguousarray(F, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    assert F.shape == (9, ny, nx) and L.shape == (ny, nx)
    _check(lib().ifdlbm_set_state(h.ptr, cav, _dptr(F), _dptr(L)))


def ifdlbm_status(h: Handle, cav: int) -> int:
    return _check(lib().ifdlbm_status(h.ptr, cav))


def ifdlbm_info(h: Handle) -> dict:
    i = ifdlbm_info_t()
    _check(lib().ifdlbm_info(h.ptr, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in ifdlbm_info_t._fields_}


IFDLBM_OBJ_KINETIC_ENERGY = 0


def ifdlbm_gradient(cavity: Cavity, options: Optional[ifdlbm_options] = None, n_steps: int = 1,
                    objective: int = IFDLBM_OBJ_KINETIC_ENERGY):
    """(J, [dJ/dtheta_rad, dJ/dn, dJ/du_lid]) of the objective after n_steps steps."""
    options = options or ifdlbm_default_options()
    J = ctypes.c_double()
    grad = np.zeros(3)
    _check(lib().ifdlbm_gradient(ctypes.byref(cavity.c()), ctypes.byref(options), int(n_steps), int(objective),
                                 ctypes.byref(J), _dptr(grad)))
    return J.value, grad


def ifdlbm_gradient_noalloc(cavity: Cavity, options: Optional[ifdlbm_options] = None, n_steps: int = 1,
                            objective: int = IFDLBM_OBJ_KINETIC_ENERGY):
    """ifdlbm_gradient with its work arrays in the library's per-GPU scratch array (no device allocation)."""
    options = options or ifdlbm_default_options()
    J = ctypes.c_double()
    grad = np.zeros(3)
    _check(lib().ifdlbm_gradient_noalloc(ctypes.byref(cavity.c()), ctypes.byref(options), int(n_steps),
                                         int(objective), ctypes.byref(J), _dptr(grad)))
    return J.value, grad


def ifdlbm_adjoint(cavity: Cavity, options: Optional[ifdlbm_options] = None, n_steps: int = 1,
                   checkpoint_every: int = 500, objective: int = IFDLBM_OBJ_KINETIC_ENERGY):
    """(J, [dJ/dtheta_rad, dJ/dn, dJ/du_lid]) by the checkpointed discrete adjoint."""
    options = options or ifdlbm_default_options()
    J = ctypes.c_double()
    grad = np.zeros(3)
    _check(lib().ifdlbm_adjoint(ctypes.byref(cavity.c()), ctypes.byref(options), int(n_steps), int(checkpoint_every),
                                int(objective), ctypes.byref(J), _dptr(grad)))
    return J.value, grad


def ifdlbm_autotune(h: Handle, steps_per_trial: int = 20):
    """(segment rows chosen, ms per step) of the fused kernel's tile-shape autotuner."""
    rows, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().ifdlbm_autotune(h.ptr, steps_per_trial, ctypes.byref(rows), ctypes.byref(ms)))
    return rows.value, ms.value


def ifdlbm_record(h: Handle, every: int, capacity: int = 0) -> None:
    _check(lib().ifdlbm_record(h.ptr, every, capacity))


def ifdlbm_get_record(h: Handle, cav: int, max_samples: int = 1 << 20):
    """(steps, u, v, ke) of the recorded samples of cavity cav, oldest first."""
    n = ctypes.c_int32(0)
    steps = np.zeros(max_samples, dtype=np.int64)
    u, v, ke = (np.zeros(max_samples) for _ in range(3))
    _check(lib().ifdlbm_get_record(h.ptr, cav, max_samples, ctypes.byref(n),
                                   steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(u), _dptr(v), _dptr(ke)))
    m = n.value
    return steps[:m].copy(), u[:m].copy(), v[:m].copy(), ke[:m].copy()


def ifdlbm_time_step(h: Handle, cav: int) -> float:
    dt = ctypes.c_double(0.0)
    _check(lib().ifdlbm_time_step(h.ptr, cav, ctypes.byref(dt)))
    return dt.value


def ifdlbm_classify(x, dt_sample: float, steady_tol: float = 1e-6) -> dict:
    a = np.ascontiguousarray(x, dtype=np.float64)
    r = ifdlbm_regime_t()
    _check(lib().ifdlbm_classify(_dptr(a), a.size, dt_sample, steady_tol, ctypes.byref(r)))
    out = {f[0]: getattr(r, f[0]) for f in ifdlbm_regime_t._fields_}
    out["name"] = REGIMES[r.regime]
    return out


def ifdlbm_destroy(h: Handle) -> None:
    h.close()


def ifdlbm_strerror(code: int) -> str:
    return _strerror(code)


def ifdlbm_last_error() -> str:
    return lib().ifdlbm_last_error().decode()


def ifdlbm_build_digest() -> str:
    """SHA-256 of the sources the loaded library was built from."""
    return lib().ifdlbm_build_digest().decode()
