"""Pins of the mixed-quadrature (App. A) oracle for the spatially homogeneous
gas, against what the mathematics fixes independently of its code:
  - the product rule integrates products of 1-D polynomials exactly;
  - the factorised equilibrium of order N_a >= 2 carries the point's n, u
    and T (App. A.2), and is a fixed point of the right-hand side at F = 0;
  - the force term's moments are the exact sources 0, n F_a, n F.u
    (App. A.3 with the per-axis identity of Sec. IV.B.4);
  - a homogeneous gas under a constant force keeps n and T and drifts with
    u(t) = u0 + F t, exactly (BGK conserves n, u, T and RK-3 integrates the
    linear and quadratic moment histories without error);
  - a negative control: the half-range force without its delta term
    (Eq. deltaf) loses mass."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import multi as M

SETS = {
    "HH(4)xH(4)": [M.Axis(O.HALF, 4, 3), M.Axis(O.FULL, 4, 3)],
    "HH(3)xHH(3)xH(4)": [M.Axis(O.HALF, 3, 2), M.Axis(O.HALF, 3, 2), M.Axis(O.FULL, 4, 3)],
    "H(6)xHH(4,p0=1.2)xL(3)": [M.Axis(O.FULL, 6, 5), M.Axis(O.HALF, 4, 3, 1.2),
                                M.Axis(O.LAGUERRE, 3, 2, 0.6)],
}


def _state(axes, npts, seed):
    """Positive populations: a product equilibrium times a seeded positive
    modulation (rough in p on purpose: the identities hold for any f)."""
    rng = np.random.default_rng(seed)
    n = 1.0 + 0.3 * rng.random(npts)
    u = 0.2 * (rng.random((npts, len(axes))) - 0.5)
    T = 0.8 + 0.5 * rng.random(npts)
    f = M.feq(axes, n, u, T) * (1.0 + 0.1 * rng.random((npts, M.nodes(axes)[0].shape[1])))
    return f


@pytest.mark.parametrize("name", list(SETS))
def test_product_rule_exactness(name):
    """sum_v W_v prod_a p_a^{s_a} = prod_a mu_a(s_a) for s_a <= 2 Q_a - 1:
    each factor a 1-D moment of its axis' normalised weight."""
    axes = SETS[name]
    P, W = M.nodes(axes)
    assert P.shape == (len(axes), W.size)
    # the weights of the product are products: their sum is the product of the
    # per-axis sums (1 for Hermite axes, 2 for a Laguerre one, 1 per half)
    sums = [O.tables(ax.quad, ax.Q, ax.p0)[1].sum() for ax in axes]
    assert np.isclose(W.sum(), np.prod(sums), rtol=1e-14)

    def mu(ax, s):
        p, w, *_ = O.tables(ax.quad, ax.Q, ax.p0)
        return float(np.sum(w * p ** s))
    for s in [(0, 1, 2), (2, 2, 0), (1, 3, 1), (3, 0, 2)]:
        s = s[:len(axes)]
        got = np.sum(W * np.prod([P[a] ** s[a] for a in range(len(axes))], axis=0))
        ref = np.prod([mu(ax, s[a]) for a, ax in enumerate(axes)])
        assert abs(got - ref) < 1e-14 * max(1.0, abs(ref))
    # the x index is the slowest: the first V_y V_z nodes share p_x
    Vrest = W.size // axes[0].V
    assert np.all(P[0, :Vrest] == P[0, 0])


@pytest.mark.parametrize("name", list(SETS))
def test_equilibrium_moments_and_fixed_point(name):
    axes = SETS[name]
    rng = np.random.default_rng(1)
    n = 1.0 + rng.random(5)
    u = 0.3 * (rng.random((5, len(axes))) - 0.5)
    T = 0.7 + rng.random(5)
    f = M.feq(axes, n, u, T)
    n2, u2, T2 = M.moments(axes, f)
    np.testing.assert_allclose(n2, n, rtol=1e-13)
    np.testing.assert_allclose(u2, u, rtol=0, atol=1e-13)
    np.testing.assert_allclose(T2, T, rtol=1e-13)
    L = M.rhs(axes, f, np.zeros(len(axes)), 0.3)
    assert np.abs(L).max() < 1e-13 * np.abs(f).max()


@pytest.mark.parametrize("name", list(SETS))
def test_force_term_moments(name):
    """sum_v L = 0, sum_v p_a L = n F_a, sum_v |p|^2/2 L = n F.u for the pure
    force term on an arbitrary positive state."""
    axes = SETS[name]
    f = _state(axes, 6, 2)
    F = np.array([0.7, -1.3, 0.4])[:len(axes)]
    L = M.rhs(axes, f, F, math.inf)
    P, _ = M.nodes(axes)
    n, u, T = M.moments(axes, f)
    sc = np.abs(f).sum(axis=1)
    np.testing.assert_allclose(L.sum(axis=1), 0, atol=1e-13 * sc.max())
    np.testing.assert_allclose(L @ P.T, n[:, None] * F[None, :], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose((L * (P ** 2).sum(axis=0)).sum(axis=1) / 2, n * (u @ F), rtol=1e-12,
                               atol=1e-13)


@pytest.mark.parametrize("name", list(SETS))
@pytest.mark.parametrize("Kn", [math.inf, 0.2])
def test_homogeneous_drift(name, Kn):
    """n and T stay, u(t) = u0 + F t after 40 RK-3 steps."""
    axes = SETS[name]
    f = _state(axes, 3, 3)
    F = np.array([0.5, -0.25, 0.8])[:len(axes)]
    dt, nsteps = 2e-3, 40
    n0, u0, T0 = M.moments(axes, f)
    y = M.run(axes, f, F, Kn, dt, nsteps)
    n1, u1, T1 = M.moments(axes, y)
    np.testing.assert_allclose(n1, n0, rtol=1e-13)
    np.testing.assert_allclose(u1, u0 + F[None, :] * dt * nsteps, rtol=0, atol=1e-13)
    np.testing.assert_allclose(T1, T0, rtol=1e-12)
    # not vacuous: the populations do change
    assert np.abs(y - f).max() > 1e-3 * np.abs(f).max()


def test_force_without_delta_term_loses_mass():
    """Negative control: the half-range K with the delta-term part removed
    (Eq. deltaf) breaks the zero-mass source on the x axis."""
    axes = SETS["HH(4)xH(4)"]
    f = _state(axes, 2, 4)
    _, _, K, _, Kd = O.tables(O.HALF, 4)
    Vx, Vy = axes[0].V, axes[1].V
    fr = f.reshape(2, Vx, Vy)
    Kf = np.tensordot(K - Kd, fr, axes=([1], [1]))
    assert np.abs(Kf.sum(axis=0)).max() > 1e-3 * np.abs(fr).max()
