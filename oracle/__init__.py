"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the serial FP64 CPU oracle.

The oracle (``ifdlbm_oracle.c``) is a plain implementation of the IFDLBM of
arXiv:2306.07603 for the lid-driven isosceles-trapezoid cavity, written from
the paper.  Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package; the GPU library never does, and
this package never imports the GPU library.

State layout: ``F`` is ``(9, ny, nx)`` float64 (the distribution f-hat of
Eq. 2.3), ``Lam`` is ``(ny, nx)`` float64 (the relaxation time that produced
it).  Equation numbers are the paper's labels.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ifdlbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CAVITY, COUETTE, PERIODIC = 0, 1, 2
DT_CONTRAVARIANT, DT_CARTESIAN = 0, 1
LAMBDA_LAGGED, LAMBDA_IMPLICIT = 0, 1


def compile_source(src: str, out: str, defines=()) -> str:
    """gcc -O2 -ffp-contract=off, serial FP64: the oracle's only build recipe (defines: -D options, such as
    ORC_COMPLEX_STEP for the complex-step build)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call([
        "gcc", "-O2", "-ffp-contract=off", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra",
        *["-D" + d for d in defines], "-I", _HERE, "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library in place, and its complex-step build."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    from . import complex_step
    complex_step.build(force)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("re", ctypes.c_double),
                ("n", ctypes.c_double), ("theta_deg", ctypes.c_double), ("u_lid", ctypes.c_double),
                ("cfl", ctypes.c_double), ("mix", ctypes.c_double), ("rho0", ctypes.c_double),
                ("gamma_min", ctypes.c_double), ("bc_mode", ctypes.c_int), ("dt_rule", ctypes.c_int),
                ("lambda_mode", ctypes.c_int)]


class _Derived(ctypes.Structure):
    _fields_ = [("dxi", ctypes.c_double), ("deta", ctypes.c_double), ("dt", ctypes.c_double),
                ("K", ctypes.c_double), ("cot", ctypes.c_double), ("lam0", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def load(path: str):
    """Load an oracle library built by compile_source and declare its calls."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(_Params)
    L.orc_derive.argtypes = [P, ctypes.POINTER(_Derived)]
    L.orc_lattice.argtypes = [_D, _D, _D, _D, _D]
    L.orc_equilibrium.argtypes = [ctypes.c_double] * 4 + [_D]
    L.orc_moments.argtypes = [_D, ctypes.c_double, _D, _D, _D]
    L.orc_node_xy.argtypes = [P, ctypes.c_int, ctypes.c_int, _D, _D]
    L.orc_contravariant.argtypes = [P, ctypes.c_int, ctypes.c_int, _D, _D, _D]
    L.orc_stream_term.argtypes = [P, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.orc_stream_term.restype = ctypes.c_double
    L.orc_init.argtypes = [P, _D, _D]
    L.orc_run.argtypes = [P, _D, _D, ctypes.c_long, _D, _D]
    L.orc_fields.argtypes = [P, _D, _D, _D, _D]
    L.orc_f_from_fhat.argtypes = [P, _D, _D, _D]
    L.orc_kinetic_energy.argtypes = [P, _D]
    L.orc_kinetic_energy.restype = ctypes.c_double
    L.orc_residuals.argtypes = [P, _D, _D, _D, _D, _D]
    L.orc_f_from_fhat_node.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, _D]
    L.orc_f_from_fbar.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, _D]
    L.orc_collide.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, _D, _D]
    L.orc_relaxation_time.argtypes = [_D, _D] + [ctypes.c_double] * 5
    L.orc_relaxation_time.restype = ctypes.c_double
    L.orc_relaxation_time_implicit.argtypes = [_D, _D] + [ctypes.c_double] * 4
    L.orc_relaxation_time_implicit.restype = ctypes.c_double
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB)
    return _lib


@contextlib.contextmanager
def using(path: str):
    """Temporarily route every call of this module to another oracle build."""
    global _lib
    saved = lib()
    _lib = load(path)
    try:
        yield
    finally:
        _lib = saved


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


@dataclass
class Params:
    """Problem parameters (Eq. 1.4, 1.5, 2.15.1, 3.8.1) and solver options."""
    nx: int = 33
    ny: int = 33
    re: float = 100.0
    n: float = 1.0
    theta_deg: float = 90.0
    u_lid: float = 0.1
    cfl: float = 0.5
    mix: float = 0.75
    rho0: float = 1.0
    gamma_min: float = 1e-6
    bc_mode: int = CAVITY
    dt_rule: int = DT_CONTRAVARIANT
    lambda_mode: int = LAMBDA_LAGGED

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.re, self.n, self.theta_deg, self.u_lid, self.cfl,
                       self.mix, self.rho0, self.gamma_min, self.bc_mode, self.dt_rule, self.lambda_mode)


def derive(p: Params) -> dict:
    d = _Derived()
    rc = lib().orc_derive(ctypes.byref(p.c()), ctypes.byref(d))
    if rc != 0:
        raise ValueError("parameters outside the method's domain: %r" % (p,))
    return {k: getattr(d, k) for k, _ in _Derived._fields_}


def lattice():
    cx, cy, w, wb = (np.zeros(9) for _ in range(4))
    cs2 = ctypes.c_double()
    lib().orc_lattice(_ptr(cx), _ptr(cy), _ptr(w), _ptr(wb), ctypes.byref(cs2))
    return cx, cy, w, wb, cs2.value


def equilibrium(P: float, ux: float, uy: float, rho0: float = 1.0) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_equilibrium(P, ux, uy, rho0, _ptr(out))
    return out


def moments(f: np.ndarray, rho0: float = 1.0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    P, ux, uy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_moments(_ptr(f), rho0, ctypes.byref(P), ctypes.byref(ux), ctypes.byref(uy))
    return P.value, ux.value, uy.value


def f_from_fhat_node(fh, feq, lam: float, dt: float) -> np.ndarray:
    fh, feq, out = np.ascontiguousarray(fh, float), np.ascontiguousarray(feq, float), np.zeros(9)
    lib().orc_f_from_fhat_node(_ptr(fh), _ptr(feq), lam, dt, _ptr(out))
    return out


def f_from_fbar(fb, feq, lam: float, dt: float) -> np.ndarray:
    fb, feq, out = np.ascontiguousarray(fb, float), np.ascontiguousarray(feq, float), np.zeros(9)
    lib().orc_f_from_fbar(_ptr(fb), _ptr(feq), lam, dt, _ptr(out))
    return out


def collide(fh, feq, lam: float, dt: float):
    fh, feq = np.ascontiguousarray(fh, float), np.ascontiguousarray(feq, float)
    fhp, fbp = np.zeros(9), np.zeros(9)
    lib().orc_collide(_ptr(fh), _ptr(feq), lam, dt, _ptr(fhp), _ptr(fbp))
    return fhp, fbp


def relaxation_time(fh, feq, lam_old: float, dt: float, K: float, n: float, gamma_min: float) -> float:
    fh, feq = np.ascontiguousarray(fh, float), np.ascontiguousarray(feq, float)
    return lib().orc_relaxation_time(_ptr(fh), _ptr(feq), lam_old, dt, K, n, gamma_min)


def relaxation_time_implicit(fh, feq, dt: float, K: float, n: float, gamma_min: float) -> float:
    fh, feq = np.ascontiguousarray(fh, float), np.ascontiguousarray(feq, float)
    return lib().orc_relaxation_time_implicit(_ptr(fh), _ptr(feq), dt, K, n, gamma_min)


def node_xy(p: Params, i: int, j: int):
    x, y = ctypes.c_double(), ctypes.c_double()
    lib().orc_node_xy(ctypes.byref(p.c()), i, j, ctypes.byref(x), ctypes.byref(y))
    return x.value, y.value


def contravariant(p: Params, i: int, j: int):
    cxi, ceta, J = np.zeros(9), np.zeros(9), ctypes.c_double()
    lib().orc_contravariant(ctypes.byref(p.c()), i, j, _ptr(cxi), _ptr(ceta), ctypes.byref(J))
    return cxi, ceta, J.value


def stream_term(p: Params, Phi: np.ndarray, k: int, i: int, j: int) -> float:
    Phi = np.ascontiguousarray(Phi, dtype=np.float64)
    assert Phi.shape == (9, p.ny, p.nx)
    return lib().orc_stream_term(ctypes.byref(p.c()), _ptr(Phi), k, i, j)


def init(p: Params):
    F = np.zeros((9, p.ny, p.nx))
    Lam = np.zeros((p.ny, p.nx))
    if lib().orc_init(ctypes.byref(p.c()), _ptr(F), _ptr(Lam)) != 0:
        raise ValueError("bad parameters %r" % (p,))
    return F, Lam


def run(p: Params, F: np.ndarray, Lam: np.ndarray, nsteps: int):
    """Advance (F, Lam) in place by nsteps; returns (E(u), E(P)) of the last step."""
    ru, rp = ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_run(ctypes.byref(p.c()), _ptr(F), _ptr(Lam), int(nsteps), ctypes.byref(ru), ctypes.byref(rp))
    if rc == -1:
        raise ValueError("bad parameters %r" % (p,))
    if rc == -2:
        raise FloatingPointError("oracle state became non-finite")
    return ru.value, rp.value


def residuals(p: Params, F_old: np.ndarray, F_new: np.ndarray):
    """Eq. (2.19) between two states: (E(u), E(P), E(P) with the mean of P removed)."""
    eu, ep, eg = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_residuals(ctypes.byref(p.c()), _ptr(np.ascontiguousarray(F_old)), _ptr(np.ascontiguousarray(F_new)),
                        ctypes.byref(eu), ctypes.byref(ep), ctypes.byref(eg))
    return eu.value, ep.value, eg.value


def fields(p: Params, F: np.ndarray):
    u, v, P = (np.zeros((p.ny, p.nx)) for _ in range(3))
    lib().orc_fields(ctypes.byref(p.c()), _ptr(F), _ptr(u), _ptr(v), _ptr(P))
    return u, v, P


def f_from_fhat(p: Params, F: np.ndarray, Lam: np.ndarray) -> np.ndarray:
    f = np.zeros_like(F)
    lib().orc_f_from_fhat(ctypes.byref(p.c()), _ptr(F), _ptr(Lam), _ptr(f))
    return f


def kinetic_energy(p: Params, F: np.ndarray) -> float:
    return lib().orc_kinetic_energy(ctypes.byref(p.c()), _ptr(F))


def simulate(p: Params, nsteps: int):
    """Step (1) then nsteps of Steps (2)-(8); returns (u, v, P, F, Lam)."""
    F, Lam = init(p)
    if nsteps:
        run(p, F, Lam, nsteps)
    u, v, P = fields(p, F)
    return u, v, P, F, Lam
