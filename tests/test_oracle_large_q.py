"""Pins of the oracle's large-Q half-range Gauss-Hermite construction (the
three-term recurrence from a discretised Stieltjes procedure, Sturm
bisection for the nodes, Eq. wk_half_gen for the weights), used above Q = 16
and needed for the paper's HHLB(20;200) runs (Sec. V.E).  Checked against
the monomial construction where both apply, and against what the weight
fixes at any Q: exactness against the Gamma-function moments, the
force-moment identity, mass conservation and the equilibrium's half-range
moments (independent 40-50 digit arithmetic)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O


def mu_half(s):
    """int_0^inf z^s exp(-z^2/2)/sqrt(2 pi) dz."""
    return mp.mpf(2) ** (mp.mpf(s) / 2) * mp.gamma((s + 1) / mp.mpf(2)) / (2 * mp.sqrt(mp.pi))


@pytest.fixture
def recurrence_everywhere():
    old = O.set_qmono(0)
    yield
    O.set_qmono(old)


@pytest.mark.parametrize("Q", [1, 2, 4, 8, 12, 16])
def test_recurrence_construction_matches_monomial_one(Q, recurrence_everywhere):
    """Where both constructions apply, they give the same rule, force matrix
    and equilibrium (the monomial one is pinned in test_oracle_pins.py)."""
    p, w, K, Kin, Kd = O.tables(O.HALF, Q)
    g = O.equilibrium(O.HALF, Q, Q - 1, 1.1, 0.17, 1.3)
    old = O.set_qmono(32)
    try:
        pm, wm, Km, Kinm, Kdm = O.tables(O.HALF, Q)
        gm = O.equilibrium(O.HALF, Q, Q - 1, 1.1, 0.17, 1.3)
    finally:
        O.set_qmono(old)
    np.testing.assert_allclose(p, pm, rtol=1e-15)
    np.testing.assert_allclose(w, wm, rtol=1e-14)
    np.testing.assert_allclose(K, Km, rtol=0, atol=2e-15 * np.abs(Km).max())
    np.testing.assert_allclose(Kd, Kdm, rtol=0, atol=2e-15 * np.abs(Kdm).max())
    np.testing.assert_allclose(g, gm, rtol=0, atol=2e-15 * np.abs(gm).max())


@pytest.mark.parametrize("Q", [17, 40, 100, 200, 256])
def test_large_q_quadrature_exact_to_degree_2Q_minus_1(Q):
    """Sec. IV.B.1: exactness for z^s, s <= 2Q-1 (every s up to 40, then
    every 7th, and 2Q-1), to the rounding of the FP64 table (node rounding
    grows with s through z^s).  At Q = 17 degree 2Q is visibly not exact; at
    larger Q its truncation error is already below rounding."""
    mp.mp.dps = 40
    p, w, *_ = O.tables(O.HALF, Q)
    z, wz = [mp.mpf(x) for x in p[:Q]], [mp.mpf(x) for x in w[:Q]]
    assert np.all(np.diff(p[:Q]) > 0) and p[0] > 0
    assert np.all(p[:Q] < 2.5 * math.sqrt(Q))          # Fig. (hh_hyp) envelope
    ss = sorted(set(list(range(min(41, 2 * Q))) + list(range(41, 2 * Q, 7)) + [2 * Q - 1]))
    for s in ss:
        got = mp.fsum(a * b ** s for a, b in zip(wz, z))
        assert abs(got / mu_half(s) - 1) < 3e-15 + 2e-17 * s, (Q, s)
    if Q < 20:
        got = mp.fsum(a * b ** (2 * Q) for a, b in zip(wz, z))
        assert abs(got / mu_half(2 * Q) - 1) > 1e-13


def _moment_identity_error(p, K, s, cols):
    worst = mp.mpf(0)
    for kp in cols:
        terms = [mp.mpf(p[k]) ** s * mp.mpf(K[k, kp]) for k in range(len(p))]
        lhs = mp.fsum(terms)
        rhs = -s * mp.mpf(p[kp]) ** (s - 1) if s > 0 else mp.mpf(0)
        scale = mp.fsum(abs(t) for t in terms) + abs(rhs)
        worst = max(worst, abs(lhs - rhs) / scale)
    return float(worst)


def _gauss_recurrence(n):
    """Monic recurrence pi_{k+1} = (z - alpha_k) pi_k - beta_k pi_{k-1} of the
    half-range weight, from its exact moments mu_s (Gamma function) by the
    classical Chebyshev algorithm in mp.dps digits.  The algorithm is
    ill-conditioned: at n = 257 it needs about 330 digits."""
    mu = [mu_half(s) for s in range(2 * n)]
    alpha, beta = [mp.mpf(0)] * n, [mp.mpf(0)] * n
    sig_m, sig = [mp.mpf(0)] * (2 * n), list(mu)
    alpha[0], beta[0] = mu[1] / mu[0], mu[0]
    for k in range(1, n):
        new = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_m[l]
        alpha[k] = new[k + 1] / new[k] - sig[k] / sig[k - 1]
        beta[k] = new[k] / sig[k - 1]
        sig_m, sig = sig, new
    return alpha, beta


def test_large_q_nodes_are_gauss_roots():
    """Sec. IV.B.1 at Q = 256, the largest half-range order: every node is a
    root of the degree-Q orthogonal polynomial of the half-range weight, that
    polynomial taken from the exact moments (not from the oracle's own
    discretised Stieltjes procedure): the Newton step pi_Q / pi_Q' at each
    node is below 1e-15 of the node.  (Moment exactness cannot decide this:
    at Q = 256 node sets 1e-9 apart reproduce every moment to 1e-14.)"""
    Q = 256
    mp.mp.dps = 400
    alpha, beta = _gauss_recurrence(Q + 1)
    p, *_ = O.tables(O.HALF, Q)
    worst = 0.0
    for z in p[:Q]:
        z = mp.mpf(z)
        pm, pc, dm, dc = mp.mpf(0), mp.mpf(1), mp.mpf(0), mp.mpf(0)
        for k in range(Q):
            pn = (z - alpha[k]) * pc - (beta[k] * pm if k > 0 else 0)
            dn = pc + (z - alpha[k]) * dc - (beta[k] * dm if k > 0 else 0)
            pm, pc, dm, dc = pc, pn, dc, dn
        worst = max(worst, float(abs(pc / dc / z)))
    assert worst < 1e-15, worst


@pytest.mark.parametrize("Q", [40, 200])
def test_large_q_force_matrix_moments_and_mass(Q):
    """Sec. IV.B.4: sum_k p_k^s K_kk' = -s p_k'^{s-1} for s < Q (sampled s and
    columns from both halves), and zero column sums (mass)."""
    mp.mp.dps = 40
    p, w, K, Kin, Kd = O.tables(O.HALF, Q)
    V = 2 * Q
    cols = sorted(set([0, 1, Q // 2, Q - 1, Q, Q + 1, Q + Q // 2, V - 1]))
    for s in sorted(set([0, 1, 2, 3, 5, 10, Q // 2, Q - 1])):
        assert _moment_identity_error(p, K, s, cols) < 1e-13, s
    colabs = np.abs(K).sum(axis=0)
    assert np.max(np.abs(K.sum(axis=0)) / colabs) < 1e-14
    assert np.max(np.abs((K - Kd).sum(axis=0)) / colabs) > 1e-6


@pytest.mark.parametrize("Q,N", [(40, 20), (200, 20)])
def test_large_q_equilibrium_half_range_moments(Q, N):
    """Sec. IV.B.3: half-range moments s <= N of g_k equal the Maxwellian's."""
    mp.mp.dps = 30
    u, T = 0.13, 1.6
    g = O.equilibrium(O.HALF, Q, N, 1.0, u, T)
    p, *_ = O.tables(O.HALF, Q)
    maxw = lambda x: mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
    gp = [mp.mpf(x) for x in g]
    pp = [mp.mpf(x) for x in p]
    for s in range(N + 1):
        ref_p = mp.quad(lambda x: x ** s * maxw(x), [0, mp.inf])
        ref_m = mp.quad(lambda x: (-x) ** s * maxw(-x), [0, mp.inf])
        got_p = mp.fsum(gp[k] * pp[k] ** s for k in range(Q))
        got_m = mp.fsum(gp[k] * pp[k] ** s for k in range(Q, 2 * Q))
        sc = mp.quad(lambda x: abs(x) ** s * maxw(x), [-mp.inf, mp.inf])
        assert abs(got_p - ref_p) / sc < 1e-13, s
        assert abs(got_m - ref_m) / sc < 1e-13, s
    with pytest.raises(ValueError):     # the recurrence rules keep orders N <= 20
        O.equilibrium(O.HALF, Q, 21, 1.0, u, T)


# ---------------------------------------------------------------- full range

@pytest.fixture
def full_recurrence_everywhere():
    old = O.set_qfmono(0)
    yield
    O.set_qfmono(old)


@pytest.mark.parametrize("Q", [2, 8, 20, 40, 64])
def test_full_range_recurrence_matches_monomial(Q, full_recurrence_everywhere):
    """Where both full-range constructions apply (Q <= 64), the recurrence
    one (Sturm roots, Eqs. H_wk and H_Kk through h_l = He_l / sqrt(l!)) gives
    the monomial one's rule and force matrix."""
    p, w, K, *_ = O.tables(O.FULL, Q)
    old = O.set_qfmono(64)
    try:
        pm, wm, Km, *_ = O.tables(O.FULL, Q)
    finally:
        O.set_qfmono(old)
    np.testing.assert_allclose(p, pm, rtol=2e-15, atol=1e-15)
    np.testing.assert_allclose(w, wm, rtol=1e-14)
    colmax = np.abs(Km).max(axis=0)
    assert np.max(np.abs(K - Km) / colmax) < 1e-14


@pytest.mark.parametrize("Q", [100, 150])
def test_full_range_large_q_matches_numpy_hermegauss(Q):
    """Sec. IV.A.1: the nodes are the roots of He_Q; with the normalised
    weight the weights are numpy's hermegauss weights / sqrt(2 pi)."""
    p, w, *_ = O.tables(O.FULL, Q)
    xs, ws = np.polynomial.hermite_e.hermegauss(Q)
    ws = ws / math.sqrt(2 * math.pi)
    order = np.argsort(p)
    np.testing.assert_allclose(p[order], xs, rtol=0, atol=1e-13)
    live = ws > 1e-250
    np.testing.assert_allclose(w[order][live], ws[live], rtol=1e-11)


@pytest.mark.parametrize("Q", [100, 500])
def test_full_range_large_q_exactness_and_force_moments(Q):
    """Exactness against the Gaussian moments (s-1)!! to degree 2Q-1
    (sampled), the force-moment identity sum_k p_k^s K_kk' = -s p_k'^{s-1}
    for s < Q (sampled s and columns), and zero column sums relative to each
    column's size (Sec. IV.A.4)."""
    mp.mp.dps = 40
    p, w, K, *_ = O.tables(O.FULL, Q)
    z, wz = [mp.mpf(x) for x in p], [mp.mpf(x) for x in w]
    for s in sorted(set([0, 1, 2, 3, 4, 10, 40, Q, 2 * Q - 2, 2 * Q - 1])):
        got = mp.fsum(a * b ** s for a, b in zip(wz, z))
        ref = mp.mpf(0) if s % 2 else mp.fac2(s - 1)
        scale = mp.fsum(a * abs(b) ** s for a, b in zip(wz, z))
        assert abs(got - ref) / scale < 3e-15 + 2e-17 * s, s
    cols = sorted(set([0, 1, Q // 4, Q // 2 - 1, Q // 2, Q - 1]))
    for s in sorted(set([0, 1, 2, 5, 20, Q // 2, Q - 1])):
        worst = mp.mpf(0)
        for kp in cols:
            terms = [mp.mpf(p[k]) ** s * mp.mpf(K[k, kp]) for k in range(Q)]
            lhs = mp.fsum(terms)
            rhs = -s * mp.mpf(p[kp]) ** (s - 1) if s > 0 else mp.mpf(0)
            worst = max(worst, abs(lhs - rhs) / (mp.fsum(abs(t) for t in terms) + abs(rhs)))
        assert worst < 1e-14, s
    assert np.max(np.abs(K.sum(axis=0)) / np.abs(K).sum(axis=0)) < 1e-15


@pytest.mark.parametrize("Q", [100, 200])
def test_full_range_large_q_equilibrium_moments(Q):
    """Sec. IV.A.3: the moments s <= N of the order-N equilibrium equal the
    Maxwellian's (mpmath quadrature), and N <= 20 is enforced above Q = 64."""
    mp.mp.dps = 30
    N, u, T = 20, 0.13, 1.6
    g = O.equilibrium(O.FULL, Q, N, 1.0, u, T)
    p, *_ = O.tables(O.FULL, Q)
    maxw = lambda x: mp.exp(-(x - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
    for s in range(N + 1):
        ref = mp.quad(lambda x: x ** s * maxw(x), [-mp.inf, u, mp.inf])
        sc = mp.quad(lambda x: abs(x) ** s * maxw(x), [-mp.inf, 0, mp.inf])
        got = mp.fsum(mp.mpf(a) * mp.mpf(b) ** s for a, b in zip(g, p))
        assert abs(got - ref) / sc < 1e-13, s
    with pytest.raises(ValueError):
        O.equilibrium(O.FULL, Q, 21, 1.0, u, T)
