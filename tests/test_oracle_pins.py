"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's own formulas: each test checks a property
the paper states (exactness, moment identities, closed forms, printed tables)
or a textbook/library result, so that a dropped term, a wrong sign, index or
transposed operand in the oracle fails at least one of them.
"""
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 50


def mu_half(s):
    """int_0^inf z^s exp(-z^2/2)/sqrt(2 pi) dz = 2^{s/2} Gamma((s+1)/2) / (2 sqrt(pi))."""
    return mp.mpf(2) ** (mp.mpf(s) / 2) * mp.gamma((s + 1) / mp.mpf(2)) / (2 * mp.sqrt(mp.pi))


# ---------------------------------------------------------------- quadrature

@pytest.mark.parametrize("Q", [1, 2, 3, 4, 6, 8, 12, 16])
def test_half_range_quadrature_exact_to_degree_2Q_minus_1(Q):
    """Sec. IV.B.1: the Q-point half-range rule integrates z^s exactly for s <= 2Q-1."""
    p, w, *_ = O.tables(O.HALF, Q)
    z, wz = p[:Q], w[:Q]
    assert np.all(np.diff(z) > 0) and np.all(z > 0)
    for s in range(2 * Q):
        got = mp.fsum(mp.mpf(wk) * mp.mpf(zk) ** s for wk, zk in zip(wz, z))
        assert abs(got / mu_half(s) - 1) < 3e-15, (Q, s)
    # not vacuous: degree 2Q is no longer exact
    got = mp.fsum(mp.mpf(wk) * mp.mpf(zk) ** (2 * Q) for wk, zk in zip(wz, z))
    assert abs(got / mu_half(2 * Q) - 1) > 1e-13


def test_half_range_q1_closed_form():
    """Q = 1: h_1 root z = mu_1/mu_0 = sqrt(2/pi), weight mu_0 = 1/2."""
    p, w, K, *_ = O.tables(O.HALF, 1)
    assert p[0] == pytest.approx(math.sqrt(2 / math.pi), rel=1e-15)
    assert p[1] == -p[0]
    assert w[0] == pytest.approx(0.5, rel=1e-15)
    # Eq. (hh_Kk_hh) with Q = 1: only the cross term survives,
    # K = (w sigma_k/p0) (-1/(2 sqrt(2 pi))) Phi_0^2 with Phi_0 = h_{0,0}^2 = 2.
    ref = np.array([[-1.0, -1.0], [1.0, 1.0]]) / math.sqrt(2 * math.pi)
    np.testing.assert_allclose(K, ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("Q", [2, 4, 6, 8, 12, 16])
def test_full_range_rule_matches_library_gauss_hermite(Q):
    """Sec. IV.A.1: nodes are roots of He_Q; with the normalised weight the
    weights are numpy's hermegauss weights / sqrt(2 pi)."""
    p, w, *_ = O.tables(O.FULL, Q)
    xs, ws = np.polynomial.hermite_e.hermegauss(Q)
    ws = ws / math.sqrt(2 * math.pi)
    order = np.argsort(p)
    np.testing.assert_allclose(p[order], xs, rtol=0, atol=2e-14)
    np.testing.assert_allclose(w[order], ws, rtol=1e-12, atol=0)


def test_full_range_small_worked_cases():
    """Sec. IV.A.2: eigenvalues of the moment matrix are 0 (Q=1), +-1 (Q=2),
    0, +-sqrt(3) (Q=3)."""
    p, *_ = O.tables(O.FULL, 2)
    np.testing.assert_allclose(np.sort(p), [-1, 1], atol=1e-15)
    with pytest.raises(ValueError):   # odd Q is avoided by the paper (Sec. IV.A.1)
        O.tables(O.FULL, 3)


@pytest.mark.parametrize("Q", [1, 2, 4, 8, 12, 16])
def test_node_envelopes(Q):
    """Figs. (H_hyp)/(hh_hyp): |z| < 2 sqrt(Q) (full range), < 2.5 sqrt(Q) (half range)."""
    p, *_ = O.tables(O.HALF, Q)
    assert np.all(np.abs(p) < 2.5 * math.sqrt(Q))
    if Q % 2 == 0:
        pf, *_ = O.tables(O.FULL, Q)
        assert np.all(np.abs(pf) < 2 * math.sqrt(Q))


# ------------------------------------------------------------- force matrix

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


@pytest.mark.parametrize("quad,Q", [(O.HALF, 1), (O.HALF, 2), (O.HALF, 4), (O.HALF, 8),
                                    (O.HALF, 16), (O.FULL, 4), (O.FULL, 16)])
def test_force_matrix_moments(quad, Q):
    """Sec. IV.B.4: moments s < Q of the discrete momentum derivative are exact,
    sum_k p_k^s K_kk' = -s p_k'^{s-1}: s = 0 is mass (the delta term), s = 1
    the momentum source nF, s = 2 the energy source nFu."""
    p, w, K, *_ = O.tables(quad, Q)
    for s in range(Q):
        assert _moment_identity_error(p, K, s) < 2e-15, s
    if Q > 1:  # not vacuous: order Q is not reproduced
        assert _moment_identity_error(p, K, Q + 1) > 1e-10


@pytest.mark.parametrize("quad,Q", [(O.HALF, 4), (O.HALF, 8), (O.HALF, 16), (O.FULL, 8)])
@pytest.mark.parametrize("p0", [1.0, 1.3])
def test_force_matrix_differentiates_reference_maxwellian(quad, Q, p0):
    """The Maxwellian with T = p0^2/m, u = 0 has f_k = w_k and
    d/dp f = -(p/p0^2) f, which the force matrix reproduces exactly."""
    p, w, K, *_ = O.tables(quad, Q, p0)
    np.testing.assert_allclose(K @ w, -(p / p0 ** 2) * w, rtol=1e-12, atol=1e-15 * w.max())


@pytest.mark.parametrize("Q", [1, 2, 4, 8])
def test_negative_control_no_delta_term(Q):
    """Sec. I and Eq. (hh_dftheta): the per-half derivative alone (within-half
    term plus its boundary term, Eq. dfpm) changes the mass: its column sums
    are -sigma_k' omega(0) Phi_0(|z_k'|)/p0, i.e. the bias f(0+) - f(0-) of
    Eq. (dtn_hemi).  Adding the delta term (Eq. deltaf_full) cancels it."""
    p, w, K, Kin, Kd = O.tables(O.HALF, Q)
    no_delta = K - Kd
    assert np.max(np.abs(no_delta.sum(axis=0))) > 0.1
    assert np.max(np.abs(K.sum(axis=0))) < 1e-13 * np.abs(K).max()
    # the delta term is a rank-1 block coupling the halves
    assert np.linalg.matrix_rank(Kd, tol=1e-12 * np.abs(Kd).max()) == 1
    assert np.abs(Kd[:Q, Q:]).max() > 0
    # the within-half sum term does not couple the two halves (theta(p p'), Eq. hh_K)
    assert np.all(Kin[:Q, Q:] == 0) and np.all(Kin[Q:, :Q] == 0)
    # a distribution continuous at p = 0 in the sense f(0+) = f(0-) -- here the
    # discrete Maxwellian at rest -- is differentiated identically with or
    # without the delta term (its coefficient f^+(0) - f^-(0) vanishes)
    np.testing.assert_allclose(Kd @ w, 0, atol=1e-15)


# --------------------------------------------------------------- equilibrium

@pytest.mark.parametrize("Q", [3, 4, 8, 12, 16])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.1, 1.5), (-0.2, 2.0), (0.05, 0.7), (0.3, 1.2)])
def test_equilibrium_reproduces_n_u_T(Q, u, T):
    """N >= 2: the discrete equilibrium has density n, velocity u, temperature T."""
    n = 1.7
    g = O.equilibrium(O.HALF, Q, Q - 1, n, u, T)
    p, *_ = O.tables(O.HALF, Q)
    assert g.sum() == pytest.approx(n, rel=2e-15)
    uu = (p * g).sum() / g.sum()
    assert uu == pytest.approx(u, abs=2e-15)
    TT = ((p - uu) ** 2 * g).sum() / g.sum()
    assert TT == pytest.approx(T, rel=2e-15)


@pytest.mark.parametrize("Q,N", [(4, 3), (8, 7), (8, 4), (16, 15)])
def test_equilibrium_half_range_moments(Q, N):
    """Sec. IV.B.3: the half-range moments s <= N of g_k equal those of the
    Maxwellian (numerical integration at 50 digits, independent of the oracle)."""
    u, T = 0.13, 1.6
    g = O.equilibrium(O.HALF, Q, N, 1.0, u, T)
    p, *_ = O.tables(O.HALF, Q)
    maxw = lambda x: mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
    for s in range(N + 1):
        ref_p = mp.quad(lambda x: x ** s * maxw(x), [0, mp.inf])
        ref_m = mp.quad(lambda x: (-x) ** s * maxw(-x), [0, mp.inf])
        got_p = mp.fsum(mp.mpf(g[k]) * mp.mpf(p[k]) ** s for k in range(Q))
        got_m = mp.fsum(mp.mpf(g[k]) * mp.mpf(p[k]) ** s for k in range(Q, 2 * Q))
        sc = mp.quad(lambda x: abs(x) ** s * maxw(x), [-mp.inf, mp.inf])
        assert abs(got_p - ref_p) / sc < 1e-14, s
        assert abs(got_m - ref_m) / sc < 1e-14, s


def _hh_coeffs_mp(lmax):
    """Orthonormal half-range Hermite monomial coefficients at 50 digits."""
    mu = [mu_half(s) for s in range(2 * lmax + 2)]
    C = []
    for l in range(lmax + 1):
        v = [mp.mpf(0)] * (l + 1)
        v[l] = mp.mpf(1)
        for _ in range(2):
            for j in range(l):
                pr = mp.fsum(v[a] * C[j][b] * mu[a + b] for a in range(l + 1) for b in range(j + 1))
                for b in range(j + 1):
                    v[b] -= pr * C[j][b]
        nr = mp.sqrt(mp.fsum(v[a] * v[b] * mu[a + b] for a in range(l + 1) for b in range(l + 1)))
        C.append([x / nr for x in v])
    return C


def _poly_deriv_exp(sign, s):
    """Coefficients (ascending) of P_s^{+/-}(zeta) = e^{-+zeta^2} d^s/dzeta^s e^{+-zeta^2}:
    P_0 = 1, P_{s+1} = P_s' +- 2 zeta P_s."""
    P = [Fraction(1)]
    for _ in range(s):
        d = [Fraction(i) * P[i] for i in range(1, len(P))] + [Fraction(0), Fraction(0)]
        nxt = [Fraction(0)] * (len(P) + 1)
        for i, c in enumerate(d[:len(nxt)]):
            nxt[i] += c
        for i, c in enumerate(P):
            nxt[i + 1] += sign * 2 * c
        P = nxt
    return P


def _peval(coefs, x):
    return mp.fsum(mp.mpf(c.numerator) / c.denominator * x ** i for i, c in enumerate(coefs))


@pytest.mark.parametrize("Q", [4, 8])
def test_equilibrium_matches_printed_closed_form(Q):
    """Eq. (hh_gk) as printed (erf/exp form with P^+_s, P^*_s and Phi^N_s),
    evaluated at 50 digits, equals the oracle's equilibrium."""
    N = Q - 1
    u, T = 0.21, 1.4
    m, p0 = 1, 1
    C = _hh_coeffs_mp(N)
    p, w, *_ = O.tables(O.HALF, Q)
    zeta = u * mp.sqrt(m / (2 * mp.mpf(T)))
    Pp = [_poly_deriv_exp(+1, s) for s in range(N + 1)]
    Pm = [_poly_deriv_exp(-1, s) for s in range(N + 1)]

    def Pstar(s, x):
        return mp.fsum(mp.binomial(s, j) * _peval(Pp[j], x) * _peval(Pm[s - j - 1], x)
                       for j in range(s))

    def hval(l, z):
        return mp.fsum(C[l][i] * z ** i for i in range(l + 1))

    ref = []
    for half in (+1, -1):
        ze = half * zeta
        for k in range(Q):
            zk = mp.mpf(p[k])
            acc = mp.mpf(0)
            for s in range(N + 1):
                Phi = mp.fsum(C[l][s] * hval(l, zk) for l in range(s, N + 1))
                br = (1 + mp.erf(ze)) * _peval(Pp[s], ze) + 2 / mp.sqrt(mp.pi) * mp.exp(-ze ** 2) * Pstar(s, ze)
                acc += (m * mp.mpf(T) / (2 * p0 ** 2)) ** (mp.mpf(s) / 2) * Phi * br
            ref.append(mp.mpf(w[k]) / 2 * acc)
    got = O.equilibrium(O.HALF, Q, N, 1.0, u, T)
    ref = np.array([float(x) for x in ref])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # the smallest (tail) entries too, relative to their own size
    np.testing.assert_allclose(got, ref, rtol=1e-9)


@pytest.mark.parametrize("quad,Q", [(O.HALF, 4), (O.HALF, 16), (O.FULL, 16)])
def test_equilibrium_reference_temperature_is_weights(quad, Q):
    """At T = p0^2/m, u = 0: f_k = w_k p0 g(p_k)/omega(z_k) = w_k."""
    p, w, *_ = O.tables(quad, Q)
    g = O.equilibrium(quad, Q, Q - 1, 1.0, 0.0, 1.0)
    np.testing.assert_allclose(g, w, rtol=1e-13)


@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.2, 1.5), (-0.3, 0.8)])
def test_full_range_equilibrium_moments(u, T):
    """Eq. (H_gk) with N = Q-1 reproduces n, u, T and the full-range moments
    up to order N (Gauss-Hermite exactness, Sec. IV.A.3)."""
    Q = 16
    g = O.equilibrium(O.FULL, Q, Q - 1, 1.0, u, T)
    p, *_ = O.tables(O.FULL, Q)
    for s in range(Q):
        ref = mp.quad(lambda x: x ** s * mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T),
                      [-mp.inf, mp.inf])
        sc = mp.quad(lambda x: abs(x) ** s * mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T),
                     [-mp.inf, mp.inf])
        got = mp.fsum(mp.mpf(g[k]) * mp.mpf(p[k]) ** s for k in range(Q))
        assert abs(got - ref) / sc < 1e-13, s


# ------------------------------------------------------------------ WENO-5

def _read_weno_table():
    rows = []
    with open(os.path.join(GOLDEN, "weno_limits.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            rows.append((key, [float(Fraction(v)) for v in vals]))
    return rows


def _sigmas(a, b, c, d, e):
    """Smoothness indicators of Eq. (weno_sigma), used only to construct inputs."""
    s1 = 13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    s2 = 13 / 12 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    s3 = 13 / 12 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    return s1, s2, s3


def test_weno_limit_table():
    """Table (weno): weights when one, two or all smoothness indicators vanish.
    sigma_1 = 0 iff f_{i-2} = f_{i-1} = f_i, sigma_2 = 0 iff f_{i-1} = f_i =
    f_{i+1}, sigma_3 = 0 iff f_i = f_{i+1} = f_{i+2}."""
    stencils = {
        "equal": (1.0, 1.0, 1.0, 1.0, 1.0),
        "2,3": (5.0, 1.0, 1.0, 1.0, 1.0),
        "1,2": (1.0, 1.0, 1.0, 1.0, 7.0),
        "1": (1.0, 1.0, 1.0, 2.0, 5.0),
        "2": (4.0, 1.0, 1.0, 1.0, 3.0),
        "3": (9.0, 1.0, 2.0, 2.0, 2.0),
    }
    # sigma_1 = sigma_3 = 0 forces all five values equal (then sigma_2 = 0 as
    # well), so that row is reached only in floating point, where delta/sigma^2
    # overflows for sigma_1 and sigma_3 but not for sigma_2: a = b = c = 0,
    # e = 2.375 d with d = 6.67e-78 (sigma^2 near the overflow threshold of delta/sigma^2).
    d = 6.67e-78
    tiny = (0.0, 0.0, 0.0, d, 2.375 * d)
    s1, s2, s3 = _sigmas(*tiny)
    with np.errstate(over="ignore", divide="ignore"):
        r = np.array([0.1, 0.6, 0.3]) / np.array([s1, s2, s3]) ** 2
    assert np.isinf(r[0]) and np.isinf(r[2]) and np.isfinite(r[1])
    stencils["1,3"] = tiny
    rows = _read_weno_table()
    assert len(rows) == 7
    for key, ref in rows:
        s = _sigmas(*stencils[key])
        if key not in ("equal", "1,3"):
            zero = {int(q) for q in key.split(",")}
            assert all((s[q - 1] == 0) == (q in zero) for q in (1, 2, 3)), key
        om, _ = O.weno5(*stencils[key])
        np.testing.assert_allclose(om, ref, rtol=0, atol=1e-15, err_msg=key)
    # equal non-zero sigmas give the ideal weights as well (first row)
    om, _ = O.weno5(0.0, 1.0, 2.0, 3.0, 4.0)
    np.testing.assert_allclose(om, [0.1, 0.6, 0.3], atol=1e-15)


def test_weno_exact_for_linear_data():
    """Every WENO-5 candidate is exact for linear data, so the face value is too."""
    for slope in (0.3, -2.0):
        vals = [1.0 + slope * j for j in (-2, -1, 0, 1, 2)]
        _, face = O.weno5(*vals)
        assert face == pytest.approx(1.0 + slope * 0.5, rel=1e-15)


def _advection_error(adv, Nx):
    ch = O.Channel(quad=O.HALF, Q=2, Nx=Nx, adv=adv, Dt=0, Kn=math.inf, g=0.0, dt=1e-3)
    p, w, *_ = O.tables(O.HALF, 2)
    _, dx, xc = O.grid(ch)
    prof = 1.0 + 0.5 * np.exp(xc)          # smooth and monotone: no critical points
    dprof = 0.5 * np.exp(xc)
    f = np.ascontiguousarray(w[:, None] * prof[None, :])
    Lf, _, _ = O.rhs(ch, f, None)
    inner = slice(4, Nx - 4)
    err = 0.0
    for k in range(len(p)):
        exact = -p[k] * w[k] * dprof[inner]
        err = max(err, np.max(np.abs(Lf[k, inner] - exact)) / (abs(p[k]) * w[k]))
    return err


@pytest.mark.parametrize("adv,order", [(O.WENO5, 5), (O.UPWIND3, 3)])
def test_advection_convergence_order(adv, order):
    """Sec. IV.C.2: WENO-5 is fifth order on smooth data; the third-order
    upwind scheme third order (uniform grid, interior cells)."""
    e1, e2 = _advection_error(adv, 40), _advection_error(adv, 80)
    rate = math.log2(e1 / e2)
    assert rate > order - 0.4, rate


# ---------------------------------------------------------------- full step

def _read_butcher():
    A, b, c = [], None, []
    with open(os.path.join(GOLDEN, "rk3_butcher.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            left, right = line.split("|")
            vals = [float(Fraction(x)) for x in right.split()]
            if left.split()[0] == "b":
                b = vals
            else:
                c.append(float(Fraction(left.split()[1])))
                A.append(vals)
    return np.array(A), np.array(b), np.array(c)


def test_rk3_amplification_of_collision_mode():
    """Eq. (rk3) / Table (rk3): a spatially uniform perturbation with zero
    density, momentum and energy relaxes by the stability function of the
    printed tableau, R(z) = 1 + z b^T (I - zA)^{-1} 1, z = -dt/tau, tau = Kn/n
    (Eq. tau).  Checked in cells the walls cannot reach within one step."""
    A, b, _ = _read_butcher()
    Q, Nx, Kn, n0, dt = 4, 40, 0.05, 1.3, 0.01
    ch = O.Channel(quad=O.HALF, Q=Q, Nx=Nx, adv=O.WENO5, Dt=2, Kn=Kn, g=0.0, dt=dt)
    p, w, *_ = O.tables(O.HALF, Q)
    f, chi = O.initial_state(ch, n0=n0)
    # perturbation orthogonal to 1, p, p^2 (least-squares projection)
    rng = np.random.default_rng(7)
    d = rng.standard_normal(2 * Q) * w
    Mx = np.stack([np.ones_like(p), p, p * p])
    d = d - Mx.T @ np.linalg.solve(Mx @ Mx.T, Mx @ d)
    d *= 0.05 * n0 / np.abs(d).max()
    assert np.abs(Mx @ d).max() < 1e-15
    fp = f + d[:, None]
    f1, _, _ = O.run(ch, 1, fp, chi)
    z = -dt * n0 / Kn
    R = 1 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))
    assert R == pytest.approx(1 + z + z * z / 2 + z ** 3 / 6, rel=1e-14)
    inner = slice(10, Nx - 10)
    np.testing.assert_allclose(f1[:, inner] - f[:, inner], R * d[:, None] * np.ones((1, Nx - 20)),
                               rtol=0, atol=1e-14)


def test_rhs_moment_sources():
    """For a uniform state in the interior, the right-hand side has no mass
    source, momentum source n F and energy source n F u (the force-term
    moments; collisions conserve all three)."""
    Q, Nx, g = 8, 24, -0.37
    ch = O.Channel(quad=O.HALF, Q=Q, Nx=Nx, adv=O.WENO5, Dt=2, Kn=0.2, g=g, dt=1e-3)
    p, w, *_ = O.tables(O.HALF, Q)
    rng = np.random.default_rng(3)
    fk = w * (1 + 0.3 * rng.random(2 * Q))
    ck = w * (0.8 + 0.4 * rng.random(2 * Q))
    f = np.ascontiguousarray(np.repeat(fk[:, None], Nx, 1))
    chi = np.ascontiguousarray(np.repeat(ck[:, None], Nx, 1))
    Lf, Lc, _ = O.rhs(ch, f, chi)
    n = fk.sum()
    u = (p * fk).sum() / n
    i = Nx // 2
    assert abs(Lf[:, i].sum()) < 1e-14
    assert (p * Lf[:, i]).sum() == pytest.approx(n * g, rel=1e-13)
    energy = (0.5 * p * p * Lf[:, i]).sum() + Lc[:, i].sum()
    assert energy == pytest.approx(n * g * u, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("adv,A", [(O.UPWIND3, 0.0), (O.WENO5, 0.9)])
def test_mass_conservation_and_zero_wall_flux(adv, A):
    """Sec. IV.C.3: zero net mass flux at each wall plus the mass-conserving
    force matrix keep N = sum_i dx_i n_i constant to rounding."""
    ch = O.Channel(quad=O.HALF, Q=4, Nx=48, adv=adv, A=A, Dt=2, Kn=0.1, g=-0.5,
                   T_left=1.0, T_right=1.5, dt=2e-4)
    f, chi = O.initial_state(ch)
    _, dx, _ = O.grid(ch)
    # one right-hand side of a random positive state: mass rate vanishes
    rng = np.random.default_rng(1)
    fr = f * (1 + 0.2 * rng.random(f.shape))
    Lf, _, _ = O.rhs(ch, np.ascontiguousarray(fr), chi)
    assert abs((dx[None, :] * Lf).sum()) < 1e-13 * np.abs(dx[None, :] * Lf).sum()
    f2, c2, nw = O.run(ch, 1500, f, chi)
    n, _, _ = O.moments(ch, f2, c2)
    assert abs((dx * n).sum() - 1.0) < 2e-13
    assert np.all(nw > 0)


def test_mass_bias_without_delta_term():
    """Sec. I: dropping the delta term (a planted mistake in the oracle) makes
    the total mass drift, i.e. the cross term is what conserves it."""
    ch = O.Channel(quad=O.HALF, Q=4, Nx=32, adv=O.WENO5, Dt=2, Kn=0.1, g=-0.5,
                   T_left=1.0, T_right=1.5, dt=2e-4)
    f, chi = O.initial_state(ch)
    _, dx, _ = O.grid(ch)
    fb, cb, _ = O.run(ch, 400, f, chi, drop_delta=True)
    n, _, _ = O.moments(ch, fb, cb)
    assert abs((dx * n).sum() - 1.0) > 1e-4


def test_equal_wall_equilibrium_is_fixed_point():
    """Sec. V.B with g = 0: the uniform Maxwellian at the wall temperature is
    a steady state of the discrete step (up to rounding)."""
    ch = O.Channel(quad=O.HALF, Q=8, Nx=32, adv=O.WENO5, A=0.9, Dt=2, Kn=0.05, g=0.0,
                   T_left=1.3, T_right=1.3, dt=1e-4)
    f, chi = O.initial_state(ch, T0=1.3)
    f2, c2, nw = O.run(ch, 50, f, chi)
    np.testing.assert_allclose(f2, f, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(nw, [1.0, 1.0], rtol=1e-13)


@pytest.mark.slow
def test_barometric_profile_small_channel():
    """Sec. V.B, Eq. (iso_n) with g = -g_p: equal walls, any Kn, the steady
    density is n(x) = m g N exp(m g x/T_w) / (2 T_w sinh(m g L/(2 T_w))) with
    u = 0, T = T_w.  Half-range HHLB(3;4), N_x = 64, Kn = 0.1, g = -0.1,
    third-order upwind, dt = 5e-4, 20 000 steps (t = 10)."""
    ch = O.Channel(quad=O.HALF, Q=4, N=3, Nx=64, adv=O.UPWIND3, Dt=2, Kn=0.1, g=-0.1,
                   T_left=1.0, T_right=1.0, dt=5e-4)
    f, chi = O.initial_state(ch)
    f2, c2, _ = O.run(ch, 20000, f, chi)
    n, u, T = O.moments(ch, f2, c2)
    _, dx, xc = O.grid(ch)
    mass = (dx * n).sum()
    g, Tw, L = ch.g, 1.0, 1.0
    nref = g * mass * np.exp(g * xc / Tw) / (2 * Tw * math.sinh(g * L / (2 * Tw)))
    assert np.max(np.abs(n / nref - 1)) < 2e-4
    assert np.max(np.abs(u)) < 2e-4
    assert np.max(np.abs(T - 1)) < 2e-4


@pytest.mark.parametrize("Nx,A", [(64, 0.9), (513, 0.99), (24, 0.99), (512, 0.5)])
def test_stretched_grid_faces(Nx, A):
    """Sec. IV.C.2, Eqs. (x_eta) and (etai): the faces x(eta_{i +- 1/2}) of
    Nx cells of equal eta-width on [-artanh A, artanh A].  Pinned without the
    mapping itself: the end faces are the walls -L/2, +L/2 (tanh(artanh A) =
    A); the grid is mirror-symmetric about x = 0; the cells are coarsest at
    the centre and densest at the walls (the paper's stated purpose), widening
    monotonically towards the centre; and, since dx/deta = L/(2A) sech^2 eta,
    the width ratio wall/centre tends to 1 - A^2 as Nx grows (midpoint
    widths, checked to O(deta^2))."""
    L = 1.0
    ch = O.Channel(Q=2, Nx=Nx, A=A, L=L)
    xf, dx, xc = O.grid(ch)
    assert xf[0] == pytest.approx(-L / 2, abs=2e-16) and xf[-1] == pytest.approx(L / 2, abs=2e-16)
    np.testing.assert_allclose(xf, -xf[::-1], rtol=0, atol=4e-16)
    np.testing.assert_allclose(dx, dx[::-1], rtol=4e-13, atol=0)
    np.testing.assert_allclose(np.diff(xf), dx, rtol=1e-12, atol=0)
    assert abs(dx.sum() - L) < 1e-14
    half = dx[: (Nx + 1) // 2]
    assert np.all(np.diff(half) > 0), "cells must widen from the wall towards the centre"
    assert dx.argmin() in (0, Nx - 1)
    deta = 2.0 / Nx * math.atanh(A)
    centre = L / (2 * A) * deta            # dx at eta = 0 to O(deta^3)
    wall = centre * (1 - A * A)            # dx at eta = +-artanh A to first order
    # the wall cell's own midpoint sits deta/2 inside the wall: sech^2 there
    eta_w = math.atanh(A) - deta / 2
    assert dx[0] == pytest.approx(centre / math.cosh(eta_w) ** 2, rel=deta ** 2)
    assert dx[0] / dx.max() == pytest.approx(1 - A * A, rel=3 * deta + deta ** 2 * 50)
    assert wall > 0


def test_uniform_grid_when_unstretched():
    """A = 0: Nx equal cells of width L/Nx between the walls."""
    for Nx, L in ((64, 1.0), (17, 2.5)):
        xf, dx, xc = O.grid(O.Channel(Q=2, Nx=Nx, A=0.0, L=L))
        np.testing.assert_allclose(dx, L / Nx, rtol=1e-14)
        np.testing.assert_allclose(xc, 0.5 * (xf[1:] + xf[:-1]), atol=1e-15)
        assert xf[0] == pytest.approx(-L / 2) and xf[-1] == pytest.approx(L / 2)
