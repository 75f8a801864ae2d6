"""GPU parity of the mixed-quadrature velocity space (App. A) for the
spatially homogeneous gas: hhlb_multi_rhs and hhlb_multi_step through the C
ABI against the numpy oracle (oracle/multi.py), element by element, and the
exact drift invariants (n and T constant, u = u0 + F t) at a size the
oracle does not reach.

Tolerance: 1e-12 of the point's scale, the FP64 bar of the 1-D path.  The
scale of L at a point is max_v |L_v| plus max_v |f_v| n / Kn (the BGK term's
size), so a right-hand side in which force and relaxation nearly cancel is
still held to the size of its terms."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle as O  # noqa: E402
from oracle import multi as M  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12

# (name, [(quad, Q, N, p0)], F)
SETS = [
    ("HH(4)xH(4)", [(0, 4, 3, 1.0), (1, 4, 3, 1.0)], [0.7, -1.3]),
    ("HH(3)xHH(3)xH(4)", [(0, 3, 2, 1.0), (0, 3, 2, 1.0), (1, 4, 3, 1.0)], [0.5, -0.25, 0.8]),
    ("H(6)xHH(4,p0=1.2)xL(3,p0=0.6)", [(1, 6, 5, 1.0), (0, 4, 3, 1.2), (2, 3, 2, 0.6)], [-0.4, 0.9, 0.3]),
    ("HH(8)xH(8)xH(4), V = 512", [(0, 8, 7, 1.0), (1, 8, 7, 1.0), (1, 4, 3, 1.0)], [0.2, 0.1, -0.6]),
    ("HH(2)xL(3,p0=0.6)xH(4), V = 96", [(0, 2, 1, 1.0), (2, 3, 2, 0.6), (1, 4, 3, 1.0)], [0.4, -0.7, 0.2]),
    ("HH(12)xH(4), N = 11, V = 96", [(0, 12, 11, 1.0), (1, 4, 3, 1.0)], [0.6, -0.3]),
    ("HH(10)xH(10)xH(2), N = 9, V = 400", [(0, 10, 9, 1.0), (1, 10, 9, 1.0), (1, 2, 1, 1.0)], [-0.2, 0.5, 0.3]),
]
# sets with V <= 128 run four points per wave (16 lanes each), larger ones one;
# sets with every N_a <= 7 run the kernel with 8-entry coefficient arrays,
# the last two the one with 21


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _axes(spec):
    import paper_1708_03249_amd as H
    return ([H.Axis(q, Q, N, p0) for q, Q, N, p0 in spec],
            [M.Axis({0: O.HALF, 1: O.FULL, 2: O.LAGUERRE}[q], Q, N, p0) for q, Q, N, p0 in spec])


def _state(oaxes, npts, seed):
    rng = np.random.default_rng(seed)
    n = 1.0 + 0.3 * rng.random(npts)
    u = 0.25 * (rng.random((npts, len(oaxes))) - 0.5)
    T = 0.7 + 0.6 * rng.random(npts)
    V = M.nodes(oaxes)[0].shape[1]
    return M.feq(oaxes, n, u, T) * (1.0 + 0.1 * rng.random((npts, V)))


@pytest.mark.parametrize("name,spec,F", SETS, ids=[s[0] for s in SETS])
@pytest.mark.parametrize("Kn", [math.inf, 0.3])
def test_multi_rhs_against_oracle(name, spec, F, Kn):
    import torch
    import paper_1708_03249_amd as H
    haxes, oaxes = _axes(spec)
    npts = 37                                    # ragged: not a multiple of the 4 points per block
    print(f"[multi] rhs {name}, Kn={Kn}, {npts} points", flush=True)
    f = _state(oaxes, npts, 11)
    ref = M.rhs(oaxes, f, np.array(F), Kn)
    s = H.MultiSolver(haxes, npts, F, Kn)
    fd = torch.from_numpy(f).cuda()
    Ld = torch.empty_like(fd)
    s.rhs(fd, Ld)
    torch.cuda.synchronize()
    L = Ld.cpu().numpy()
    n = f.sum(axis=1)
    scale = np.abs(ref).max(axis=1) + (np.abs(f).max(axis=1) * n / Kn if math.isfinite(Kn) else 0)
    err = np.max(np.abs(L - ref) / scale[:, None])
    assert err < TOL, err


@pytest.mark.parametrize("name,spec,F", SETS[:3] + SETS[4:], ids=[s[0] for s in SETS[:3] + SETS[4:]])
def test_multi_step_against_oracle(name, spec, F):
    import torch
    import paper_1708_03249_amd as H
    haxes, oaxes = _axes(spec)
    npts, dt, nsteps, Kn = 13, 2e-3, 10, 0.2
    print(f"[multi] step {name}, {npts} points x {nsteps} steps", flush=True)
    f = _state(oaxes, npts, 12)
    ref = M.run(oaxes, f, np.array(F), Kn, dt, nsteps)
    s = H.MultiSolver(haxes, npts, F, Kn)
    fd = torch.from_numpy(f).cuda()
    s.step(fd, dt, 4)
    s.step(fd, dt, nsteps - 4)                  # two calls: the workspace is reused
    torch.cuda.synchronize()
    g = fd.cpu().numpy()
    err = np.max(np.abs(g - ref) / np.abs(ref).max(axis=1, keepdims=True))
    assert err < TOL, err


def test_multi_drift_invariants_at_scale():
    """1 000 000 points of HH(4)xH(4)xH(4), the size and launch shape the
    benchmark times: after 50 RK-3 steps every point keeps n and T and
    drifts by F t (the exact solution of the moment equations), and sampled
    points (the first, one inside, the last) match the oracle."""
    import torch
    import paper_1708_03249_amd as H
    spec = [(0, 4, 3, 1.0), (1, 4, 3, 1.0), (1, 4, 3, 1.0)]
    haxes, oaxes = _axes(spec)
    F, Kn, dt, nsteps, npts = np.array([0.3, -0.2, 0.5]), 0.1, 1e-3, 50, 1_000_000
    print(f"[multi] invariants: {npts} points x {nsteps} steps", flush=True)
    rng = np.random.default_rng(5)
    base = _state(oaxes, 64, 13)
    f = base[rng.integers(0, 64, npts)] * (1.0 + 0.05 * rng.random((npts, 1)))
    P, _ = M.nodes(oaxes)
    Pt = torch.from_numpy(P).cuda()

    def mom(x):
        n = x.sum(dim=1)
        u = (x @ Pt.T) / n[:, None]
        c2 = ((Pt[None, :, :] - u[:, :, None]) ** 2).sum(dim=1)
        return n, u, (x * c2).sum(dim=1) / (3 * n)
    fd = torch.from_numpy(f).cuda()
    n0, u0, T0 = mom(fd)
    s = H.MultiSolver(haxes, npts, F, Kn)
    s.step(fd, dt, nsteps)
    torch.cuda.synchronize()
    n1, u1, T1 = mom(fd)
    assert torch.isfinite(fd).all()
    assert ((n1 - n0).abs() / n0).max().item() < 1e-13
    Ft = torch.from_numpy(F * dt * nsteps).cuda()
    assert (u1 - u0 - Ft[None, :]).abs().max().item() < 1e-13
    assert ((T1 - T0).abs() / T0).max().item() < 1e-12
    for j in (0, 123_457, npts - 1):
        ref = M.run(oaxes, f[j:j + 1], F, Kn, dt, nsteps)
        got = fd[j:j + 1].cpu().numpy()
        assert np.max(np.abs(got - ref)) < TOL * np.abs(ref).max(), j


@pytest.mark.parametrize("spec", [[(0, 4, 3, 1.0), (1, 4, 3, 1.0)],
                                  [(0, 8, 7, 1.0), (1, 8, 7, 1.0), (1, 4, 3, 1.0)]],
                         ids=["V = 32, four points per wave", "V = 512, one point per wave"])
def test_multi_single_point_and_empty(spec):
    """npts = 1 (a wave with one valid point) against the oracle, and
    npts = 0 (nothing launched, the state untouched)."""
    import torch
    import paper_1708_03249_amd as H
    haxes, oaxes = _axes(spec)
    F = np.array([0.3, -0.5, 0.2])[:len(spec)]
    f = _state(oaxes, 1, 21)
    ref = M.rhs(oaxes, f, F, 0.4)
    s = H.MultiSolver(haxes, 1, F, 0.4)
    fd = torch.from_numpy(f).cuda()
    Ld = torch.full_like(fd, float("nan"))
    s.rhs(fd, Ld)
    torch.cuda.synchronize()
    scale = np.abs(ref).max() + np.abs(f).max() * f.sum() / 0.4
    assert np.max(np.abs(Ld.cpu().numpy() - ref)) < TOL * scale
    s0 = H.MultiSolver(haxes, 0, F, 0.4)
    empty = torch.empty((0, f.shape[1]), dtype=torch.float64, device="cuda")
    s0.step(empty, 1e-3, 3)
    s0.rhs(empty, empty)
    torch.cuda.synchronize()
