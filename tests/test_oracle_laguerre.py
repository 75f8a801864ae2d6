"""Pins of the oracle's half-range Gauss-Laguerre model (Sec. IV.B with
omega(z) = exp(-z), Eqs. wk_half and hh_Kk_L) against what the paper and the
mathematics fix: numpy's Gauss-Laguerre rule, exactness against the moments
s! of exp(-z), closed forms at Q = 1 and 2, the moment identities of the
discrete derivative, the derivative of the Laplace distribution (the
Laguerre analogue of the reference Maxwellian), and the half-range moments of
the equilibrium (independent 50-digit integration)."""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O

mp.mp.dps = 50
QS = [1, 2, 3, 4, 6, 8, 12, 16]


@pytest.mark.parametrize("Q", QS)
def test_laguerre_rule_matches_numpy_laggauss(Q):
    """Sec. IV.B.1 with phi_l = L_l: nodes are the roots of L_Q and Eq. (wk_half)
    gives the Gauss-Laguerre weights (numpy's laggauss)."""
    p, w, *_ = O.tables(O.LAGUERRE, Q)
    x, wx = np.polynomial.laguerre.laggauss(Q)
    np.testing.assert_allclose(p[:Q], x, rtol=2e-15)
    np.testing.assert_allclose(w[:Q], wx, rtol=5e-14)
    np.testing.assert_array_equal(p[Q:], -p[:Q])
    np.testing.assert_array_equal(w[Q:], w[:Q])


@pytest.mark.parametrize("Q", QS)
def test_laguerre_quadrature_exact_to_degree_2Q_minus_1(Q):
    """Eq. (hh_quad): sum_k w_k z_k^s = int_0^inf exp(-z) z^s dz = s! for s <= 2Q-1."""
    p, w, *_ = O.tables(O.LAGUERRE, Q)
    z, wz = p[:Q], w[:Q]
    for s in range(2 * Q):
        got = mp.fsum(mp.mpf(wk) * mp.mpf(zk) ** s for wk, zk in zip(wz, z))
        assert abs(got / mp.factorial(s) - 1) < 1e-14 * (1 + s), (Q, s)
    got = mp.fsum(mp.mpf(wk) * mp.mpf(zk) ** (2 * Q) for wk, zk in zip(wz, z))
    assert abs(got / mp.factorial(2 * Q) - 1) > 1e-10


def test_laguerre_small_closed_forms():
    """Q = 1: L_1 = 1 - z, node 1, weight 1; only the cross term of Eq. (hh_Kk_L)
    survives, K = (w sigma_k/p0) (-1/2) Phi_0^2 with Phi_0 = L_0 = 1.
    Q = 2: nodes 2 -+ sqrt(2), weights (2 +- sqrt(2))/4."""
    p, w, K, *_ = O.tables(O.LAGUERRE, 1)
    assert p[0] == 1.0 and p[1] == -1.0 and w[0] == 1.0
    np.testing.assert_allclose(K, [[-0.5, -0.5], [0.5, 0.5]], rtol=0, atol=1e-16)
    p, w, *_ = O.tables(O.LAGUERRE, 2, p0=0.7)
    r2 = math.sqrt(2)
    np.testing.assert_allclose(p[:2], [0.7 * (2 - r2), 0.7 * (2 + r2)], rtol=1e-15)
    np.testing.assert_allclose(w[:2], [(2 + r2) / 4, (2 - r2) / 4], rtol=1e-15)


def _moment_identity_error(p, K, s):
    V = len(p)
    worst = mp.mpf(0)
    for kp in range(V):
        terms = [mp.mpf(p[k]) ** s * mp.mpf(K[k, kp]) for k in range(V)]
        lhs = mp.fsum(terms)
        rhs = -s * mp.mpf(p[kp]) ** (s - 1) if s > 0 else mp.mpf(0)
        scale = mp.fsum(abs(t) for t in terms) + abs(rhs)
        worst = max(worst, abs(lhs - rhs) / scale)
    return float(worst)


@pytest.mark.parametrize("Q", [1, 2, 4, 8, 16])
def test_laguerre_force_matrix_moments(Q):
    """Sec. IV.B.4: sum_k p_k^s K_kk' = -s p_k'^{s-1} for s < Q (mass, momentum
    and energy sources among them); order Q+1 is not reproduced."""
    p, w, K, *_ = O.tables(O.LAGUERRE, Q)
    for s in range(Q):
        assert _moment_identity_error(p, K, s) < 5e-15, s
    if Q > 1:
        assert _moment_identity_error(p, K, Q + 1) > 1e-10


@pytest.mark.parametrize("Q", [2, 4, 8, 16])
@pytest.mark.parametrize("p0", [1.0, 0.35])
def test_laguerre_force_matrix_differentiates_laplace_distribution(Q, p0):
    """f(p) = exp(-|p|/p0)/(2 p0) has f_k = w_k p0 f(p_k)/omega(z_k) = w_k/2 and
    df/dp = -sign(p) f/p0.  It is continuous at p = 0, so the delta term
    contributes nothing."""
    p, w, K, Kin, Kd = O.tables(O.LAGUERRE, Q, p0)
    sgn = np.sign(p)
    np.testing.assert_allclose(K @ w, -sgn * w / p0, rtol=1e-11, atol=1e-14 * np.abs(K).max() * w.max())
    np.testing.assert_allclose(Kd @ w, 0, atol=1e-14 * np.abs(Kd).max() * w.max())


@pytest.mark.parametrize("Q", [1, 2, 4, 8, 16])
def test_laguerre_delta_term_conserves_mass(Q):
    """Eq. (hh_Kk_L): the cross term makes every column of K sum to zero (mass);
    without the delta term's share of it the columns do not (Eq. dtn_hemi)."""
    p, w, K, Kin, Kd = O.tables(O.LAGUERRE, Q)
    colabs = np.abs(K).sum(axis=0)
    assert np.max(np.abs(K.sum(axis=0)) / colabs) < 1e-15
    assert np.max(np.abs((K - Kd).sum(axis=0)) / colabs) > 1e-3
    assert np.all(Kin[:Q, Q:] == 0) and np.all(Kin[Q:, :Q] == 0)


@pytest.mark.parametrize("Q", [3, 4, 8, 16])
@pytest.mark.parametrize("u,T,p0", [(0.0, 1.0, 0.3), (0.1, 1.5, 0.25), (-0.2, 0.8, 0.2)])
def test_laguerre_equilibrium_reproduces_n_u_T(Q, u, T, p0):
    """N >= 2: density n, velocity u and temperature T of the discrete
    equilibrium are exact."""
    n = 1.3
    g = O.equilibrium(O.LAGUERRE, Q, Q - 1, n, u, T, p0)
    p, *_ = O.tables(O.LAGUERRE, Q, p0)
    assert g.sum() == pytest.approx(n, rel=1e-14)
    uu = (p * g).sum() / g.sum()
    assert uu == pytest.approx(u, abs=1e-14)
    TT = ((p - uu) ** 2 * g).sum() / g.sum()
    assert TT == pytest.approx(T, rel=1e-14)


@pytest.mark.parametrize("Q,N,p0", [(4, 3, 0.4), (8, 7, 0.3), (8, 4, 0.3), (16, 15, 0.2)])
def test_laguerre_equilibrium_half_range_moments(Q, N, p0):
    """Sec. IV.B.3: half-range moments s <= N of g_k equal the Maxwellian's
    (50-digit numerical integration, independent of the oracle)."""
    u, T = 0.13, 1.6
    g = O.equilibrium(O.LAGUERRE, Q, N, 1.0, u, T, p0)
    p, *_ = O.tables(O.LAGUERRE, Q, p0)
    maxw = lambda x: mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
    for s in range(N + 1):
        ref_p = mp.quad(lambda x: x ** s * maxw(x), [0, mp.inf])
        ref_m = mp.quad(lambda x: (-x) ** s * maxw(-x), [0, mp.inf])
        got_p = mp.fsum(mp.mpf(g[k]) * mp.mpf(p[k]) ** s for k in range(Q))
        got_m = mp.fsum(mp.mpf(g[k]) * mp.mpf(p[k]) ** s for k in range(Q, 2 * Q))
        sc = mp.quad(lambda x: abs(x) ** s * maxw(x), [-mp.inf, mp.inf])
        assert abs(got_p - ref_p) / sc < 1e-13, s
        assert abs(got_m - ref_m) / sc < 1e-13, s


def _poly_deriv_exp(sign, s):
    """P_s^{+/-}(zeta) = e^{-+zeta^2} d^s/dzeta^s e^{+-zeta^2}: P_0 = 1, P_{s+1} = P_s' +- 2 zeta P_s."""
    P = [Fraction(1)]
    for _ in range(s):
        nxt = [Fraction(0)] * (len(P) + 1)
        for i in range(1, len(P)):
            nxt[i - 1] += i * P[i]
        for i, c in enumerate(P):
            nxt[i + 1] += sign * 2 * c
        P = nxt
    return P


def _peval(coefs, x):
    return mp.fsum(mp.mpf(c.numerator) / c.denominator * x ** i for i, c in enumerate(coefs))


@pytest.mark.parametrize("Q,p0", [(4, 0.5), (8, 0.3)])
def test_laguerre_equilibrium_matches_printed_closed_form(Q, p0):
    """Eq. (hh_gk) as printed ('irrespective of the choice of quadrature'), with
    Phi^N_s of Eq. (Phi_def) built from the Laguerre coefficients
    L_{l,s} = (-1)^s binom(l, s)/s!, at 50 digits."""
    N = Q - 1
    u, T, m = 0.21, 1.4, 1
    C = [[Fraction((-1) ** s * math.comb(l, s), math.factorial(s)) for s in range(l + 1)]
         for l in range(N + 1)]
    p, w, *_ = O.tables(O.LAGUERRE, Q, p0)
    zeta = u * mp.sqrt(m / (2 * mp.mpf(T)))
    Pp = [_poly_deriv_exp(+1, s) for s in range(N + 1)]
    Pm = [_poly_deriv_exp(-1, s) for s in range(N + 1)]

    def Pstar(s, x):
        return mp.fsum(mp.binomial(s, j) * _peval(Pp[j], x) * _peval(Pm[s - j - 1], x) for j in range(s))

    def lval(l, z):
        return mp.fsum(mp.mpf(c.numerator) / c.denominator * z ** i for i, c in enumerate(C[l]))

    ref = []
    for half in (+1, -1):
        ze = half * zeta
        for k in range(Q):
            zk = mp.mpf(p[k]) / p0
            acc = mp.mpf(0)
            for s in range(N + 1):
                Phi = mp.fsum(mp.mpf(C[l][s].numerator) / C[l][s].denominator * lval(l, zk)
                              for l in range(s, N + 1))
                br = (1 + mp.erf(ze)) * _peval(Pp[s], ze) + 2 / mp.sqrt(mp.pi) * mp.exp(-ze ** 2) * Pstar(s, ze)
                acc += (m * mp.mpf(T) / (2 * mp.mpf(p0) ** 2)) ** (mp.mpf(s) / 2) * Phi * br
            ref.append(mp.mpf(w[k]) / 2 * acc)
    got = O.equilibrium(O.LAGUERRE, Q, N, 1.0, u, T, p0)
    ref = np.array([float(x) for x in ref])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_laguerre_equal_wall_equilibrium_is_fixed_point():
    """Sec. V.B with g = 0: the uniform Maxwellian at the wall temperature is a
    steady state of the discrete step for the Laguerre velocity set too."""
    ch = O.Channel(quad=O.LAGUERRE, Q=8, Nx=32, adv=O.WENO5, A=0.9, Dt=2, Kn=0.05, g=0.0,
                   T_left=1.3, T_right=1.3, p0=0.3, dt=2e-5)
    f, chi = O.initial_state(ch, T0=1.3)
    f2, c2, nw = O.run(ch, 40, f, chi)
    np.testing.assert_allclose(f2, f, rtol=1e-12, atol=1e-15 * np.abs(f).max())
    np.testing.assert_allclose(nw, [1.0, 1.0], rtol=1e-12)


def test_laguerre_mass_conservation_with_force():
    """Zero net wall flux and the mass-conserving force matrix keep
    sum_i dx_i n_i fixed with a force and unequal walls."""
    ch = O.Channel(quad=O.LAGUERRE, Q=6, Nx=24, adv=O.WENO5, A=0.5, Dt=2, Kn=0.1, g=-0.5,
                   T_left=1.0, T_right=1.6, p0=0.35, dt=3e-5)
    f, chi = O.initial_state(ch)
    _, dx, _ = O.grid(ch)
    f2, c2, _ = O.run(ch, 200, f, chi)
    n, u, T = O.moments(ch, f2, c2)
    assert abs((dx * n).sum() - 1.0) < 1e-12
    assert np.max(np.abs(u)) > 1e-4   # not vacuous: the flow has moved
