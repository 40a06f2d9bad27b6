"""TEST INFRASTRUCTURE ONLY: derivatives of the oracle's outputs by the complex step.

The same source as the oracle, compiled with ORC_COMPLEX_STEP, computes in complex doubles: with one
parameter x set to x + i h, every output O comes out as O(x) + i h O'(x) + O(h^2), and Im(O) / h is the
derivative to rounding, with no cancellation (Squire and Trapp, SIAM Review 40, 1998).  Branches (upwind
side, shear-rate floor, time-step rule) follow the real part, so the derivative is that of the branch the
real computation takes.  Used for the derivative of the kinetic energy of Eq. (5.1) after n steps from
Step (1) with respect to the top angle theta (radians), the power-law index n and the lid speed U.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import CAVITY, Params, _HERE, _SRC, compile_source

_LIB = os.path.join(_HERE, "liboracle_cs.so")
_C = ctypes.c_double * 2   # a C complex double
_P = ctypes.c_void_p


class _CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("re", _C), ("n", _C), ("theta_deg", _C), ("u_lid", _C),
                ("cfl", _C), ("mix", _C), ("rho0", _C), ("gamma_min", _C), ("bc_mode", ctypes.c_int),
                ("dt_rule", ctypes.c_int), ("lambda_mode", ctypes.c_int)]


class _CDerived(ctypes.Structure):
    _fields_ = [("dxi", _C), ("deta", _C), ("dt", _C), ("K", _C), ("cot", _C), ("lam0", _C)]


_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB, defines=("ORC_COMPLEX_STEP",))
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_derive.argtypes = [ctypes.POINTER(_CParams), ctypes.POINTER(_CDerived)]
        L.orc_init.argtypes = [ctypes.POINTER(_CParams), _P, _P]
        L.orc_run.argtypes = [ctypes.POINTER(_CParams), _P, _P, ctypes.c_long, _P, _P]
        L.orc_kinetic_energy_into.argtypes = [ctypes.POINTER(_CParams), _P, _P]
        _lib = L
    return _lib


def _cparams(p: Params, dx: dict) -> _CParams:
    """The parameters of p, each with the imaginary part dx.get(name, 0)."""
    c = _CParams()
    c.nx, c.ny, c.bc_mode, c.dt_rule, c.lambda_mode = p.nx, p.ny, p.bc_mode, p.dt_rule, p.lambda_mode
    for name in ("re", "n", "theta_deg", "u_lid", "cfl", "mix", "rho0", "gamma_min"):
        setattr(c, name, _C(getattr(p, name), dx.get(name, 0.0)))
    return c


def derive(p: Params, dx: dict) -> dict:
    """orc_derive's constants as complex numbers, with the parameters perturbed by i dx."""
    d = _CDerived()
    if lib().orc_derive(ctypes.byref(_cparams(p, dx)), ctypes.byref(d)) != 0:
        raise ValueError("parameters outside the method's domain: %r" % (p,))
    return {k: complex(getattr(d, k)[0], getattr(d, k)[1]) for k, _ in _CDerived._fields_}


def kinetic_energy(p: Params, nsteps: int, dx: dict) -> complex:
    """Eq. (5.1) after nsteps steps from Step (1) with the parameters perturbed by i dx."""
    assert p.bc_mode == CAVITY
    c = _cparams(p, dx)
    F = np.zeros((9, p.ny, p.nx), dtype=np.complex128)
    Lam = np.zeros((p.ny, p.nx), dtype=np.complex128)
    L = lib()
    if L.orc_init(ctypes.byref(c), F.ctypes.data, Lam.ctypes.data) != 0:
        raise ValueError("bad parameters %r" % (p,))
    rc = L.orc_run(ctypes.byref(c), F.ctypes.data, Lam.ctypes.data, int(nsteps), None, None)
    if rc != 0:
        raise FloatingPointError("complex-step oracle state became non-finite")
    out = _C()
    L.orc_kinetic_energy_into(ctypes.byref(c), F.ctypes.data, ctypes.byref(out))
    return complex(out[0], out[1])


def kinetic_energy_gradient(p: Params, nsteps: int, h: float = 1e-20):
    assert h <= 1e-15   # the build treats real parts of O(h^2) as exact zeros (upwind side at c = 0)
    """(J, [dJ/dtheta (radians), dJ/dn, dJ/dU]) of Eq. (5.1) after nsteps steps, by the complex step."""
    J = kinetic_energy(p, nsteps, {}).real
    g = [kinetic_energy(p, nsteps, {"theta_deg": h * 180.0 / math.pi}).imag / h,
         kinetic_energy(p, nsteps, {"n": h}).imag / h,
         kinetic_energy(p, nsteps, {"u_lid": h}).imag / h]
    return J, np.array(g)
