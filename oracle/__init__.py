"""Plain CPU oracle for the half-range Gauss-Hermite lattice Boltzmann step.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never calls it; the two share no code.

The arithmetic lives in ``hhlb_oracle.c`` (plain C, tables in __float128).
This module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hhlb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hhlb.so")

HALF, FULL, LAGUERRE = 0, 1, 2   # half-range Hermite, full-range Hermite, half-range Laguerre
WENO5, UPWIND3 = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        # a new file replaces the old one, so processes that have the library
        # loaded keep their copy
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", _SRC, "-o", tmp,
               "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Channel(ctypes.Structure):
    _fields_ = [("quad", ctypes.c_int32), ("Q", ctypes.c_int32), ("N", ctypes.c_int32),
                ("Nx", ctypes.c_int32), ("adv", ctypes.c_int32), ("Dt", ctypes.c_int32),
                ("L", ctypes.c_double), ("A", ctypes.c_double), ("Kn", ctypes.c_double),
                ("g", ctypes.c_double), ("T_left", ctypes.c_double),
                ("T_right", ctypes.c_double), ("p0", ctypes.c_double), ("dt", ctypes.c_double)]


@dataclass
class Channel:
    """One channel: quadrature kind/order, grid, Kn, force, wall temperatures."""
    quad: int = HALF
    Q: int = 4
    N: int = -1          # < 0: min(20, Q-1), the paper's choice in Sec. V
    Nx: int = 64
    adv: int = WENO5
    Dt: int = 2
    L: float = 1.0
    A: float = 0.0
    Kn: float = 0.1
    g: float = -0.1
    T_left: float = 1.0
    T_right: float = 1.0
    p0: float = 1.0
    dt: float = 5e-4

    @property
    def V(self) -> int:
        return self.Q if self.quad == FULL else 2 * self.Q

    @property
    def n_eq(self) -> int:
        return self.N if self.N >= 0 else min(20, self.Q - 1)

    def c(self) -> _Channel:
        return _Channel(self.quad, self.Q, self.n_eq, self.Nx, self.adv, self.Dt, self.L,
                        self.A, self.Kn, self.g, self.T_left, self.T_right, self.p0, self.dt)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.orc_tables_get.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp,
                                        dp, dp]
        _lib.orc_hh_coeffs.argtypes = [ctypes.c_int, dp]
        _lib.orc_equilibrium.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 4 + [dp]
        _lib.orc_weno5.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        _lib.orc_weno5.restype = None
        _lib.orc_grid.argtypes = [ctypes.POINTER(_Channel), dp, dp, dp]
        _lib.orc_rhs.argtypes = [ctypes.POINTER(_Channel), dp, dp, dp, dp, dp]
        _lib.orc_run.argtypes = [ctypes.POINTER(_Channel), ctypes.c_long, dp, dp, dp, ctypes.c_int]
        _lib.orc_moments.argtypes = [ctypes.POINTER(_Channel), dp, dp, dp, dp, dp]
        _lib.orc_set_qmono.argtypes = [ctypes.c_int]
        _lib.orc_set_qfmono.argtypes = [ctypes.c_int]
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables(quad: int, Q: int, p0: float = 1.0):
    """Return (p, w, K, K_within, K_delta) as float64 arrays."""
    V = Q if quad == FULL else 2 * Q
    p, w = np.zeros(V), np.zeros(V)
    K, Kin, Kd = np.zeros((V, V)), np.zeros((V, V)), np.zeros((V, V))
    r = lib().orc_tables_get(quad, Q, p0, _p(p), _p(w), _p(K), _p(Kin), _p(Kd))
    if r < 0:
        raise ValueError(f"oracle: bad table arguments quad={quad} Q={Q} p0={p0}")
    return p, w, K, Kin, Kd


def set_qmono(qmono: int) -> int:
    """Test-only: half-range Hermite rules with Q > qmono are built from the
    three-term recurrence instead of monomial coefficients (default 16).
    Returns the previous value."""
    return lib().orc_set_qmono(int(qmono))


def set_qfmono(qfmono: int) -> int:
    """Test-only: full-range rules with Q > qfmono are built from the
    three-term recurrence instead of the monomial Hermite evaluation
    (default 64).  Returns the previous value."""
    return lib().orc_set_qfmono(int(qfmono))


def hh_coeffs(lmax: int) -> np.ndarray:
    out = np.zeros((lmax + 1, lmax + 1))
    if lmax_check := lib().orc_hh_coeffs(lmax, _p(out)):
        raise ValueError(f"oracle: lmax {lmax} ({lmax_check})")
    return out


def equilibrium(quad: int, Q: int, N: int, n: float, u: float, T: float, p0: float = 1.0):
    V = Q if quad == FULL else 2 * Q
    out = np.zeros(V)
    if lib().orc_equilibrium(quad, Q, N, p0, n, u, T, _p(out)) < 0:
        raise ValueError("oracle: bad equilibrium arguments")
    return out


def weno5(a, b, c, d, e):
    """Weights (3,) and face value for the upwind stencil (f_{i-2} .. f_{i+2})."""
    om = np.zeros(3)
    face = ctypes.c_double()
    lib().orc_weno5(a, b, c, d, e, _p(om), ctypes.byref(face))
    return om, face.value


def grid(ch: Channel):
    xf, dx, xc = np.zeros(ch.Nx + 1), np.zeros(ch.Nx), np.zeros(ch.Nx)
    c = ch.c()
    if lib().orc_grid(ctypes.byref(c), _p(xf), _p(dx), _p(xc)):
        raise ValueError("oracle: bad grid")
    return xf, dx, xc


def initial_state(ch: Channel, n0: float = 1.0, u0: float = 0.0, T0: float = 1.0):
    """f_k = n0 g_k(u0, T0) in every cell, chi_k = (Dt/2) T0 f_k (Dt > 0)."""
    feq = equilibrium(ch.quad, ch.Q, ch.n_eq, n0, u0, T0, ch.p0)
    f = np.ascontiguousarray(np.repeat(feq[:, None], ch.Nx, axis=1))
    chi = 0.5 * ch.Dt * T0 * f if ch.Dt > 0 else np.zeros_like(f)
    return f, np.ascontiguousarray(chi)


def rhs(ch: Channel, f, chi):
    Lf, Lc, nw = np.zeros_like(f), np.zeros_like(f), np.zeros(2)
    c = ch.c()
    chi = np.ascontiguousarray(chi) if chi is not None else np.zeros_like(f)
    if lib().orc_rhs(ctypes.byref(c), _p(np.ascontiguousarray(f)), _p(chi), _p(Lf), _p(Lc), _p(nw)):
        raise ValueError("oracle: bad channel")
    return Lf, Lc, nw


def run(ch: Channel, nsteps: int, f, chi, drop_delta: bool = False):
    """Advance (f, chi) by nsteps RK-3 steps.  Returns new (f, chi, n_wall[2])."""
    f = np.array(f, dtype=np.float64, order="C")
    chi = np.array(chi if chi is not None else np.zeros_like(f), dtype=np.float64, order="C")
    nw = np.zeros(2)
    c = ch.c()
    if lib().orc_run(ctypes.byref(c), int(nsteps), _p(f), _p(chi), _p(nw), int(drop_delta)):
        raise ValueError("oracle: bad channel")
    return f, chi, nw


def moments(ch: Channel, f, chi):
    n, u, T = np.zeros(ch.Nx), np.zeros(ch.Nx), np.zeros(ch.Nx)
    c = ch.c()
    chi = np.ascontiguousarray(chi) if chi is not None else np.zeros_like(f)
    if lib().orc_moments(ctypes.byref(c), _p(np.ascontiguousarray(f)), _p(chi), _p(n), _p(u), _p(T)):
        raise ValueError("oracle: bad channel")
    return n, u, T


def cfl_dt(ch: Channel, cfl: float) -> float:
    """Time step min(cfl * min dx / max |p_k/m|, Kn/2) (the Kn/2 cap keeps the
    explicit RK-3 step inside the stability region of the BGK relaxation)."""
    p, *_ = tables(ch.quad, ch.Q, ch.p0)
    _, dx, _ = grid(ch)
    dt = cfl * dx.min() / np.abs(p).max()
    if math.isfinite(ch.Kn):
        dt = min(dt, 0.5 * ch.Kn)
    return float(dt)
