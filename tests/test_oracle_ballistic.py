"""Pins of the closed-form ballistic solution (Sec. V.D) that the ballistic
validation compares against.  Each closed form is checked against what fixes
it independently: the kinetic solution Eq. (f_bal) integrated over p at 40
digits (density, temperature, mass flux, heat flux), the stationary
collisionless Boltzmann equation with the force -m g_p checked by finite
differences, the wall conditions (half-Maxwellians at the wall temperatures),
the particle count Eq. (Ndef), and the isothermal limit Eq. (iso_n)."""
import math

import mpmath as mp
import pytest

from oracle import ballistic as B

CASES = [(0.1, 0.4, 1.6), (0.1, 1.4, 0.6), (1.0, 0.7, 1.3), (1.0, 1.4, 0.6), (1.0, 1.0, 1.0)]
XS = [-0.5, -0.41, -0.2, 0.0, 0.17, 0.38, 0.4999]


def _pmoments(x, gp, Tp, Tm, s):
    """int p^s f_bal dp, split at the discontinuity p = -m sqrt(g_p (L - 2x))."""
    edge = -mp.sqrt(gp * (1 - 2 * mp.mpf(x)))
    f = lambda p: p ** s * B.f_bal(x, p, gp=gp, Tp=Tp, Tm=Tm)
    return mp.quad(f, [-mp.inf, edge - 1, edge]) + mp.quad(f, [edge, edge + 1, mp.inf])


@pytest.mark.parametrize("gp,Tp,Tm", CASES)
def test_density_and_temperature_are_moments_of_f_bal(gp, Tp, Tm):
    """Eqs. (bal_n), (bal_temp) against Eq. (fmoms) applied to Eq. (f_bal):
    n = int f dp, n T = int p^2/m f dp (u = 0), and the mass flux vanishes."""
    mp.mp.dps = 40
    for x in XS[::2]:      # both walls' neighbourhoods and the middle
        n = _pmoments(x, gp, Tp, Tm, 0)
        j = _pmoments(x, gp, Tp, Tm, 1)
        e2 = _pmoments(x, gp, Tp, Tm, 2)
        assert abs(B.n_bal(x, gp=gp, Tp=Tp, Tm=Tm) / float(n) - 1) < 1e-13, x
        assert abs(B.T_bal(x, gp=gp, Tp=Tp, Tm=Tm) / float(e2 / n) - 1) < 1e-13, x
        assert abs(float(j)) < 1e-25


@pytest.mark.parametrize("gp,Tp,Tm", CASES[:4])
def test_heat_flux_matches_eq_bal_q(gp, Tp, Tm):
    """Eq. (bal_q): q = int p^3/(2 m^2) f dp is constant across the channel and
    equals g N (T_+ - T_-) sqrt(2m/pi) / denominator of Eq. (bal_n)."""
    mp.mp.dps = 30
    den = B._denominator(1.0, gp, 1.0, Tp, Tm)
    q_ref = gp * (Tp - Tm) * math.sqrt(2 / math.pi) / den
    for x in (-0.45, 0.0, 0.3):
        q = float(_pmoments(x, gp, Tp, Tm, 3)) / 2
        assert abs(q - q_ref) < 1e-13 * abs(q_ref), x


@pytest.mark.parametrize("gp,Tp,Tm", CASES[:4])
def test_f_bal_is_stationary_and_collisionless(gp, Tp, Tm):
    """(p/m) df/dx - m g_p df/dp = 0 away from the discontinuity: the force
    is -m g_p along x (the potential V = m g_p x), so the solver's
    acceleration g is -g_p.  Central differences at 40 digits."""
    mp.mp.dps = 40
    h = mp.mpf("1e-12")
    for x in (-0.3, 0.1, 0.35):
        edge = -math.sqrt(gp * (1 - 2 * x))
        for p in (edge - 0.7, edge - 0.1, edge + 0.05, 0.3, 1.5):
            f = lambda xx, pp: B.f_bal(xx, pp, gp=gp, Tp=Tp, Tm=Tm)
            dfx = (f(x + h, p) - f(x - h, p)) / (2 * h)
            dfp = (f(x, p + h) - f(x, p - h)) / (2 * h)
            resid = p * dfx - gp * dfp
            assert abs(resid) < mp.mpf("1e-18") * (abs(p * dfx) + abs(gp * dfp) + 1e-30), (x, p)
            # the opposite force sign leaves a residual of the size of the terms
            assert abs(p * dfx + gp * dfp) > 1e-3 * abs(gp * dfp)


@pytest.mark.parametrize("gp,Tp,Tm", CASES[:4])
def test_walls_emit_half_maxwellians(gp, Tp, Tm):
    """At x = -L/2 the particles with p > 0 follow exp(-p^2 / 2 m T_+), at
    x = +L/2 those with p < 0 follow exp(-p^2 / 2 m T_-)."""
    mp.mp.dps = 30
    for x, T, ps in ((-0.5, Tp, (0.1, 0.8, 2.0)), (0.5, Tm, (-0.1, -0.8, -2.0))):
        f0 = B.f_bal(x, ps[0], gp=gp, Tp=Tp, Tm=Tm)
        for p in ps[1:]:
            ratio = B.f_bal(x, p, gp=gp, Tp=Tp, Tm=Tm) / f0
            p2, q2 = mp.mpf(p) ** 2, mp.mpf(ps[0]) ** 2
            assert abs(ratio / mp.exp(-(p2 - q2) / (2 * mp.mpf(T))) - 1) < 1e-25


@pytest.mark.parametrize("gp,Tp,Tm", CASES)
def test_particle_count(gp, Tp, Tm):
    """Eq. (Ndef): the density integrates to N over the channel."""
    mp.mp.dps = 20
    for N in (1.0, 2.5):
        tot = mp.quad(lambda x: B.n_bal(float(x), gp=gp, Tp=Tp, Tm=Tm, N=N), [-0.5, 0, 0.5])
        assert abs(tot / N - 1) < 1e-12


@pytest.mark.parametrize("gp,T", [(0.1, 1.0), (1.0, 1.0), (1.0, 0.6), (0.37, 2.0)])
def test_isothermal_limit(gp, T):
    """T_+ = T_- = T_w: Eq. (bal_n) reduces to Eq. (iso_n),
    n = m g N / (2 T_w sinh(m g L / 2 T_w)) exp(-m g x / T_w), and T = T_w."""
    for x in XS:
        iso = gp / (2 * T * math.sinh(gp / (2 * T))) * math.exp(-gp * x / T)
        assert abs(B.n_bal(x, gp=gp, Tp=T, Tm=T) / iso - 1) < 1e-13
        assert abs(B.T_bal(x, gp=gp, Tp=T, Tm=T) / T - 1) < 1e-14


def test_error_measure():
    """Eq. (epsmax)'s measure: the deviation over the spread, the spread
    floored at 0.1."""
    assert B.eps([1.0, 1.0, 1.0], [1.0, 1.002, 0.999]) == pytest.approx(0.02)
    assert B.eps([0.0, 0.5, 1.0], [0.01, 0.5, 1.0]) == pytest.approx(0.01)
    assert B.eps([2.0, 1.0], [1.9, 1.0]) == pytest.approx(0.1)
