"""FP64 CPU oracle of the D2Q9 hybrid LBM step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it.

``hlbm_oracle.c`` holds the method (see its header for the paper passages it
follows); this module builds it with gcc and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hlbm_oracle.c")
_LIB = os.path.join(_HERE, "libhlbm_oracle.so")

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             "-std=c99"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("phi_mode", ctypes.c_int32), ("e1_centred", ctypes.c_int32),
                ("e2_off", ctypes.c_int32), ("feq_order", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("mu", ctypes.c_double), ("sigma", ctypes.c_double),
                ("sgn_eps", ctypes.c_double), ("wall_ux_lo", ctypes.c_double),
                ("wall_ux_hi", ctypes.c_double), ("wall_theta", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.POINTER(_Params)]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_init.argtypes = [ctypes.c_void_p, P, P, P, P]
        L.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_get_state.argtypes = [ctypes.c_void_p, P, P]
        L.ora_set_state.argtypes = [ctypes.c_void_p, P, P]
        L.ora_moments.argtypes = [ctypes.c_void_p, P, P, P, P, P]
        L.ora_field.argtypes = [ctypes.c_void_p, ctypes.c_char_p, P]
        L.ora_field.restype = ctypes.c_int
        L.ora_totals.argtypes = [ctypes.c_void_p, P]
        L.ora_steps.argtypes = [ctypes.c_void_p]
        L.ora_steps.restype = ctypes.c_long
        L.ora_feq.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, P]
        L.ora_f1.argtypes = [ctypes.c_double] * 6 + [ctypes.c_int, P]
        L.ora_f1_raw.argtypes = [P, ctypes.c_int, P]
        L.ora_psi.argtypes = [ctypes.c_double, ctypes.c_double, P]
        L.ora_hermite.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.ora_hermite.restype = ctypes.c_double
        L.ora_van_albada.argtypes = [ctypes.c_double, ctypes.c_double]
        L.ora_van_albada.restype = ctypes.c_double
        L.ora_entropy.argtypes = [P, P, ctypes.c_double, ctypes.c_long, P]
        L.ora_threads.argtypes = [ctypes.c_int]
        L.ora_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads(n: int = 0) -> int:
    """Threads of the oracle's OpenMP passes: n > 0 sets them; returns the
    count in effect."""
    return int(lib().ora_threads(int(n)))


def entropy_from_theta(rho, theta, gamma):
    """s = c_v ln(theta / rho^(gamma - 1)) (oracle's own closure)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    s = np.empty_like(rho)
    lib().ora_entropy(_ptr(rho), _ptr(theta), float(gamma), rho.size, _ptr(s))
    return s


def feq(rho, ux, uy, theta, order=4):
    out = np.empty(9)
    lib().ora_feq(rho, ux, uy, theta, order, _ptr(out))
    return out


def f1(a1xx, a1xy, a1yy, ux, uy, theta, order=4):
    out = np.empty(9)
    lib().ora_f1(a1xx, a1xy, a1yy, ux, uy, theta, order, _ptr(out))
    return out


def f1_raw(a1six, order=4):
    a = np.ascontiguousarray(a1six, dtype=np.float64)
    out = np.empty(9)
    lib().ora_f1_raw(_ptr(a), order, _ptr(out))
    return out


def psi(Exx, Eyy):
    out = np.empty(9)
    lib().ora_psi(Exx, Eyy, _ptr(out))
    return out


def hermite(i, idx):
    arr = (ctypes.c_int * max(1, len(idx)))(*idx)
    return lib().ora_hermite(i, len(idx), arr)


def van_albada(a, b):
    return lib().ora_van_albada(a, b)


BC = {"periodic": 0, "extrapolate": 1, "wall": 2}
PHI = {"lbm": 0, "fd": 1}


@dataclass
class OracleParams:
    nx: int
    ny: int
    gamma: float = 1.4
    prandtl: float = 0.71
    mu: float = 1e-3
    sigma: float = 0.0
    bc_x: str = "periodic"
    bc_y: str = "periodic"
    phi_mode: str = "lbm"
    e1_centred: bool = False
    e2_off: bool = False
    feq_order: int = 4
    sgn_eps: float = 1e-12
    # bc_y = "wall": velocities along x of the walls y = 0 and y = ny - 1, and
    # their temperature
    wall_ux_lo: float = 0.0
    wall_ux_hi: float = 0.0
    wall_theta: float = 1.0

    def c(self):
        return _Params(self.nx, self.ny, BC[self.bc_x], BC[self.bc_y], PHI[self.phi_mode],
                       int(self.e1_centred), int(self.e2_off), int(self.feq_order),
                       self.gamma, self.prandtl, self.mu, self.sigma, self.sgn_eps,
                       self.wall_ux_lo, self.wall_ux_hi, self.wall_theta)


class OracleSolver:
    """Plain FP64 HLBM on the CPU (Algorithm of Sec. 3.5)."""

    def __init__(self, params: OracleParams, rho, ux, uy, s=None, theta=None):
        self.p = params
        self._cp = params.c()
        self.h = lib().ora_create(ctypes.byref(self._cp))
        if not self.h:
            raise ValueError("invalid oracle parameters")
        shape = (params.ny, params.nx)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(shape)
        ux = np.ascontiguousarray(ux, dtype=np.float64).reshape(shape)
        uy = np.ascontiguousarray(uy, dtype=np.float64).reshape(shape)
        if s is None:
            s = entropy_from_theta(rho, theta, params.gamma)
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(shape)
        lib().ora_init(self.h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(s))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ora_destroy(h)
            self.h = None

    @property
    def steps(self):
        return lib().ora_steps(self.h)

    def step(self, n=1):
        lib().ora_step(self.h, int(n))
        return self

    def moments(self):
        n = self.p.nx * self.p.ny
        outs = [np.empty(n) for _ in range(5)]
        lib().ora_moments(self.h, *[_ptr(o) for o in outs])
        shape = (self.p.ny, self.p.nx)
        names = ("rho", "ux", "uy", "s", "theta")
        return {k: o.reshape(shape) for k, o in zip(names, outs)}

    def state(self):
        n = self.p.nx * self.p.ny
        F = np.empty(9 * n)
        s = np.empty(n)
        lib().ora_get_state(self.h, _ptr(F), _ptr(s))
        return F.reshape(9, self.p.ny, self.p.nx), s.reshape(self.p.ny, self.p.nx)

    def set_state(self, F, s):
        F = np.ascontiguousarray(F, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        lib().ora_set_state(self.h, _ptr(F), _ptr(s))

    def field(self, name):
        out = np.empty(self.p.nx * self.p.ny)
        if lib().ora_field(self.h, name.encode(), _ptr(out)) != 0:
            raise KeyError(name)
        return out.reshape(self.p.ny, self.p.nx)

    def totals(self):
        out = np.empty(4)
        lib().ora_totals(self.h, _ptr(out))
        return out
