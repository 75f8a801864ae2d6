"""Mixed-quadrature velocity space in d = 2 or 3 dimensions (App. A) for a
spatially homogeneous gas: the right-hand side of Eq. (boltz_multi_k)
without the advection term,

    d f_v / dt = - sum_a F_a (K_a f)_v - (f_v - feq_v) / tau,   tau = Kn / n,

on the direct-product velocity set p_v = (p_{x,i}, p_{y,j}[, p_{z,k}])
(App. A.1), with the factorised equilibrium feq = n g_x g_y [g_z] of the
point's n, u, T (App. A.2) and the force as one 1-D contraction per axis
(App. A.3), advanced by the TVD RK-3 steps of Eq. (rk3).

TEST INFRASTRUCTURE: only the tests may use this module.  The 1-D tables
(nodes, weights, K of Eqs. H_Kk / hh_Kk) and the 1-D truncated equilibria
(Eqs. H_gk / hh_gk) come from the C oracle; everything multi-dimensional is
plain numpy here.

Layout: f has shape (npts, V) with V = prod_a V_a and the velocity index
v = (i V_y + j) V_z + k (the x index slowest); m = 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import HALF, FULL, LAGUERRE, equilibrium, tables  # noqa: F401

__all__ = ["Axis", "nodes", "moments", "feq", "rhs", "run"]


@dataclass(frozen=True)
class Axis:
    quad: int       # HALF, FULL or LAGUERRE
    Q: int
    N: int          # equilibrium order on this axis
    p0: float = 1.0

    @property
    def V(self) -> int:
        return self.Q if self.quad == FULL else 2 * self.Q


def _axis(ax: Axis):
    p, w, K, *_ = tables(ax.quad, ax.Q, ax.p0)
    return p, w, K


def nodes(axes):
    """App. A.1: momenta P (d, V) and product weights W (V,)."""
    ps, ws = zip(*[_axis(a)[:2] for a in axes])
    P = np.stack([g.ravel() for g in np.meshgrid(*ps, indexing="ij")])
    W = np.ones(1)
    for w in ws:
        W = np.multiply.outer(W, w)
    return P, W.ravel()


def moments(axes, f):
    """Eq. (fmoms) in d dimensions: n = sum f, n u_a = sum p_a f,
    d n T = sum |p - u|^2 f (m = 1).  f: (npts, V)."""
    P, _ = nodes(axes)
    n = f.sum(axis=1)
    u = (f @ P.T) / n[:, None]
    d = len(axes)
    c2 = ((P[None, :, :] - u[:, :, None]) ** 2).sum(axis=1)      # (npts, V)
    T = (f * c2).sum(axis=1) / (d * n)
    return n, u, T


def feq(axes, n, u, T):
    """App. A.2: feq_v = n g_x,i g_y,j [g_z,k], each factor the 1-D
    truncated equilibrium of order N_a at (u_a, T)."""
    out = []
    for q in range(len(n)):
        g = np.ones(1)
        for a, ax in enumerate(axes):
            g = np.multiply.outer(g, equilibrium(ax.quad, ax.Q, ax.N, 1.0, u[q, a], T[q], ax.p0))
        out.append(n[q] * g.ravel())
    return np.array(out)


def force(axes, f, F):
    """App. A.3: sum_a F_a (K_a f), K_a contracting the a-th velocity index."""
    shape = (f.shape[0],) + tuple(a.V for a in axes)
    fr = f.reshape(shape)
    out = np.zeros_like(fr)
    for a, ax in enumerate(axes):
        K = _axis(ax)[2]
        Kf = np.moveaxis(np.tensordot(K, fr, axes=([1], [a + 1])), 0, a + 1)
        out += F[a] * Kf
    return out.reshape(f.shape)


def rhs(axes, f, F, Kn):
    """Right-hand side of Eq. (boltz_multi_k) without advection."""
    L = -force(axes, f, F)
    if np.isfinite(Kn):
        n, u, T = moments(axes, f)
        L -= (f - feq(axes, n, u, T)) * (n / Kn)[:, None]
    return L


def run(axes, f, F, Kn, dt, nsteps):
    """nsteps TVD RK-3 steps of Eq. (rk3)."""
    y = np.array(f, dtype=np.float64)
    for _ in range(nsteps):
        y1 = y + dt * rhs(axes, y, F, Kn)
        y2 = 0.75 * y + 0.25 * (y1 + dt * rhs(axes, y1, F, Kn))
        y = y / 3.0 + 2.0 / 3.0 * (y2 + dt * rhs(axes, y2, F, Kn))
    return y
