"""Closed-form stationary solution of the force-driven channel in the
ballistic regime (Kn = inf), Sec. V.D of the paper: the kinetic solution
Eq. (f_bal), the density Eq. (bal_n) and the temperature Eq. (bal_temp), and
the convergence measure Eq. (epsmax).

TEST INFRASTRUCTURE: only the tests may use this module.

Conventions of the paper's derivation: walls at x = -L/2 (temperature T_+,
which emits the particles with p > 0) and x = +L/2 (temperature T_-); the
potential V(x) = m g_p x, i.e. the force -m g_p along x.  The channel
parameter g of the solver and the oracle is the acceleration along x,
g = -g_p.  N is the number of particles per unit area, Eq. (Ndef).
"""
from __future__ import annotations

import math

import mpmath as mp

__all__ = ["f_bal", "n_bal", "T_bal", "eps", "eps_max"]


def _a(m, gp, L, x, T):
    """a = m g_p (L - 2x) / (2T), the exponent of Eqs. (bal_n) and (bal_temp)."""
    return m * gp * (L - 2 * x) / (2 * T)


def _denominator(m, gp, L, Tp, Tm):
    """sqrt(T_+) [e^{mgL/T_+} erfc(-sqrt(mgL/T_+)) - 1]
       + sqrt(T_-) [e^{mgL/T_-} erfc(sqrt(mgL/T_-)) - 1]   (Eq. bal_n)."""
    bp, bm = m * gp * L / Tp, m * gp * L / Tm
    return (math.sqrt(Tp) * (math.exp(bp) * math.erfc(-math.sqrt(bp)) - 1)
            + math.sqrt(Tm) * (math.exp(bm) * math.erfc(math.sqrt(bm)) - 1))


def n_bal(x, *, gp, Tp, Tm, N=1.0, L=1.0, m=1.0):
    """Eq. (bal_n): particle number density at x (g_p > 0)."""
    ap, am = _a(m, gp, L, x, Tp), _a(m, gp, L, x, Tm)
    num = (math.exp(ap) * math.erfc(-math.sqrt(ap)) / math.sqrt(Tp)
           + math.exp(am) * math.erfc(math.sqrt(am)) / math.sqrt(Tm))
    return m * gp * N * num / _denominator(m, gp, L, Tp, Tm)


def T_bal(x, *, gp, Tp, Tm, L=1.0, m=1.0):
    """Eq. (bal_temp): temperature at x."""
    ap, am = _a(m, gp, L, x, Tp), _a(m, gp, L, x, Tm)
    ep = math.exp(ap) * math.erfc(-math.sqrt(ap))
    em = math.exp(am) * math.erfc(math.sqrt(am))
    return (math.sqrt(Tp) * ep + math.sqrt(Tm) * em) / (ep / math.sqrt(Tp) + em / math.sqrt(Tm))


def f_bal(x, p, *, gp, Tp, Tm, N=1.0, L=1.0, m=1.0):
    """Eq. (f_bal) in mpmath: theta[p + m sqrt(g_p (L - 2x))] n_+ ... +
    theta[-p - m sqrt(g_p (L - 2x))] n_- ..., with n_+- from Eq. (bal_npnm) and
    the particle count N (the expressions below Eq. bal_n)."""
    x, p = mp.mpf(x), mp.mpf(p)
    gp, Tp, Tm, N, L, m = (mp.mpf(v) for v in (gp, Tp, Tm, N, L, m))
    bp, bm = m * gp * L / Tp, m * gp * L / Tm
    den = (mp.sqrt(Tp) * (mp.exp(bp) * mp.erfc(-mp.sqrt(bp)) - 1)
           + mp.sqrt(Tm) * (mp.exp(bm) * mp.erfc(mp.sqrt(bm)) - 1))
    c = 2 * m * gp * N / den                       # n_- sqrt(T_-) = n_+ sqrt(T_+) e^{-mgL/T_+}
    nm = c / mp.sqrt(Tm)
    npl = c / mp.sqrt(Tp) * mp.exp(bp)
    edge = m * mp.sqrt(gp * (L - 2 * x))
    out = mp.mpf(0)
    if p + edge > 0:
        out += npl * mp.exp(-m * gp * (L + 2 * x) / (2 * Tp)) / mp.sqrt(2 * mp.pi * m * Tp) * mp.exp(-p * p / (2 * m * Tp))
    if -p - edge > 0:
        out += nm * mp.exp(m * gp * (L - 2 * x) / (2 * Tm)) / mp.sqrt(2 * mp.pi * m * Tm) * mp.exp(-p * p / (2 * m * Tm))
    return out


def eps(M, Mref):
    """Eq. (epsmax)'s measure: max |M - M_ref| / max(max M - min M, 0.1)."""
    spread = max(max(M) - min(M), 0.1)
    return max(abs(a - b) for a, b in zip(M, Mref)) / spread


def eps_max(n, T, x, *, gp, Tp, Tm, N=1.0, L=1.0, m=1.0):
    """Eq. (epsmax): max(eps(n), eps(T)) against Eqs. (bal_n), (bal_temp) at
    the cell centres x."""
    nref = [n_bal(xi, gp=gp, Tp=Tp, Tm=Tm, N=N, L=L, m=m) for xi in x]
    Tref = [T_bal(xi, gp=gp, Tp=Tp, Tm=Tm, L=L, m=m) for xi in x]
    return max(eps(list(n), nref), eps(list(T), Tref))
