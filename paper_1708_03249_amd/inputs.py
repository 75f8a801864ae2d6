"""Seeded synthetic input generators shared by the library and the oracle
tests.  They hold none of the method's arithmetic: only random numbers and
channel parameter draws."""
from __future__ import annotations

import numpy as np


def perturbation(seed: int, shape, amplitude: float) -> np.ndarray:
    """Multiplicative positive perturbation 1 + amplitude * U[0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 1.0 + amplitude * rng.random(shape)


def smooth_modulation(seed: int, rows: int, Nx: int, amplitude: float, max_waves: int = 3) -> np.ndarray:
    """Smooth positive factors 1 + amplitude * sin(2 pi m_r (i + 1/2) / Nx + phi_r)
    of shape (rows, Nx), with m_r ~ U{1..max_waves} and phi_r ~ U[0, 2 pi)
    drawn per row (in this order).  Applied to a uniform state they give a
    resolved, non-uniform one, like a developed channel flow."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(1, max_waves + 1, rows)
    phi = rng.uniform(0.0, 2.0 * np.pi, rows)
    x = (np.arange(Nx) + 0.5) / Nx
    return 1.0 + amplitude * np.sin(2.0 * np.pi * m[:, None] * x[None, :] + phi[:, None])


def batch_draws(n_channels: int, seed: int = 0):
    """Per-channel draws of the batched workload (in this order per channel):
    Nx ~ U{64..1024}, Q ~ U{4, 8, 12}, log10 Kn ~ U[-3, 1], g ~ U[-1, 0],
    r = T_right/T_left ~ U[1, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_channels):
        Nx = int(rng.integers(64, 1025))
        Q = int(rng.choice([4, 8, 12]))
        Kn = float(10 ** rng.uniform(-3, 1))
        g = float(rng.uniform(-1, 0))
        r = float(rng.uniform(1, 2))
        out.append(dict(Nx=Nx, Q=Q, Kn=Kn, g=g, T_right=r))
    return out


def large_batch_kn(n_channels: int, seed: int = 0):
    """Kn ~ U[0.005, 0.05] per channel of the large stretched-grid workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [float(x) for x in rng.uniform(0.005, 0.05, n_channels)]
