"""Convergence sweeps of the ballistic regime (Sec. V.F, Fig. bal_err) as
batched solvers: the paper's eight ballistic cases (g_p in {0.1, 1},
Delta T in {0.6, 0.3, 0, -0.4}, Kn = inf, the 1-D gas, tanh grid A = 0.99)
advanced to the steady state and measured with Eq. (epsmax) against the
closed forms Eqs. (bal_n), (bal_temp).

  (a) HHLB(20;200) against the number of cells Nx: the paper finds the
      error falling with Nx up to Nx ~ 36 and rising beyond, where spurious
      oscillations grow with Nx at fixed Q.
  (b) HLB(N;Q) and HHLB(N;Q), N = min(20, Q - 1), at Nx = 24 against the
      number of velocities (Q for HLB, 2Q for HHLB): the HLB error falls
      much more slowly than the HHLB error.

Each sweep point is a model class or a grid of one solver: the cases of all
points advance together, one launch sequence per class."""
import math
import os
import sys
import time

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import to_oracle  # noqa: E402

import oracle as O  # noqa: E402
from oracle import ballistic as B  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [(gp, dT) for gp in (0.1, 1.0) for dT in (0.6, 0.3, 0.0, -0.4)]
T_END = 20.0        # every case is steady by t ~ 20 at Nx = 24


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _channels(H, quad, Q, Nx, dt):
    return [H.Channel(quad=quad, Q=Q, N=min(20, Q - 1), Nx=Nx, adv=H.WENO5, transverse_dof=0,
                      stretch_A=0.99, Kn=math.inf, g=-gp, T_left=1 - dT, T_right=1 + dT, dt=dt)
            for gp, dT in CASES]


def _run(H, chans, t_end, what, graph_steps=32):
    """Advance one solver of channels (all with the same dt) to t_end; return
    eps_max (Eq. epsmax) per channel, the value one tenth of the run earlier
    (a steadiness check) and the mass."""
    dt = chans[0].dt
    assert all(c.dt == dt for c in chans)
    nsteps = int(round(t_end / dt))
    s = H.Solver(chans)
    s.set_graph_steps(graph_steps)
    try:
        s.init_equilibrium()
        t0 = time.time()
        s.step(nsteps - nsteps // 10)
        e_prev = _eps(s, chans)
        s.step(nsteps // 10)
        e = _eps(s, chans)
        _, mass, bad = s.diagnostics()
        assert int(bad.cpu().item()) == 0
        mass = mass.cpu().numpy()
        print(f"[{what}] {len(chans)} channels, {nsteps} steps of dt={dt:.3g} in {time.time() - t0:.1f} s",
              flush=True)
    finally:
        s.close()
    return e, e_prev, mass


def _eps(s, chans):
    n, u, T = (a.cpu().numpy() for a in s.moments())
    out = []
    for c, ch in enumerate(chans):
        gp, Tp, Tm = -ch.g, ch.T_left, ch.T_right
        xc = O.grid(to_oracle(ch))[2]
        a0, a1 = s.cells[c], s.cells[c + 1]
        out.append(B.eps_max(n[a0:a1], T[a0:a1], xc, gp=gp, Tp=Tp, Tm=Tm))
    return np.array(out)


def _cfl_dt(H, quad, Q, Nx, cfl=1.0):
    """The time step of the grid at CFL 1 (the paper's dt = 1e-4 at Nx = 24 is
    CFL 1.15), capped at 1e-4.  The steady state solves L[y] = 0 and does not
    depend on the time step."""
    import ctypes
    ch = _channels(H, quad, Q, Nx, -cfl)[0]
    arr = (H._CChannel * 1)(ch._c())
    h = ctypes.c_void_p()
    H._check(H.lib().hhlb_create(arr, 1, 0, None, ctypes.byref(h)))
    d = np.zeros(1)
    H._check(H.lib().hhlb_time_steps(h, H._dptr(d)))
    H.lib().hhlb_destroy(h)
    return min(1e-4, float(d[0]))


def test_hhlb_200_error_against_grid_size():
    """Fig. bal_err(a): eps_max of HHLB(20;200) for Nx = 12 .. 64.  The
    worst case over the eight cases falls from Nx = 12 to a minimum at
    24 <= Nx <= 48 and rises again at the largest grid; every case meets the
    paper's 1 % criterion only near the minimum."""
    import paper_1708_03249_amd as H
    nxs = (12, 16, 24, 36, 48, 64)
    table = {}
    for group in ((12, 16, 24), (36, 48, 64)):
        dt = min(_cfl_dt(H, H.HALF_HERMITE, 200, nx) for nx in group)
        chans = [c for nx in group for c in _channels(H, H.HALF_HERMITE, 200, nx, dt)]
        e, e_prev, mass = _run(H, chans, T_END, f"HHLB(20;200) Nx {group}")
        np.testing.assert_allclose(mass, 1.0, rtol=0, atol=1e-9)
        for k, nx in enumerate(group):
            table[nx] = (e[8 * k:8 * k + 8], e_prev[8 * k:8 * k + 8])
    worst = {nx: float(table[nx][0].max()) for nx in nxs}
    for nx in nxs:
        print(f"  Nx={nx:3d}: eps_max % " + " ".join(f"{100 * x:.3f}" for x in table[nx][0])
              + f" | worst {100 * worst[nx]:.3f}", flush=True)
    best = min(worst, key=worst.get)
    assert 24 <= best <= 48, worst
    assert worst[12] > worst[best] and worst[16] > worst[best], worst
    assert worst[64] > worst[48] > worst[best], worst
    assert worst[24] < 0.01, worst


def test_hlb_vs_hhlb_error_against_velocity_count():
    """Fig. bal_err(b): at Nx = 24, eps_max of HLB(min(20,Q-1);Q) for
    Q = 40 .. 500 velocities and HHLB(min(20,Q-1);Q) for 2Q = 40 .. 400
    velocities.  Over the sweep the worst-case HHLB error falls by a far
    larger factor than the HLB error, and at every matched velocity count
    HHLB is the more accurate; only HHLB reaches 1 %."""
    import paper_1708_03249_amd as H
    hlb_q = (40, 100, 200, 500)
    hh_q = (20, 50, 100, 200)
    chans, tags = [], []
    for Q in hlb_q:
        chans += _channels(H, H.FULL_HERMITE, Q, 24, 1e-4)
        tags.append(("HLB", Q, Q))
    for Q in hh_q:
        chans += _channels(H, H.HALF_HERMITE, Q, 24, 1e-4)
        tags.append(("HHLB", Q, 2 * Q))
    e, e_prev, mass = _run(H, chans, T_END, "HLB / HHLB velocity sweep")
    np.testing.assert_allclose(mass, 1.0, rtol=0, atol=1e-9)
    worst = {}
    for k, (model, Q, V) in enumerate(tags):
        ek = e[8 * k:8 * k + 8]
        worst[(model, V)] = float(ek.max())
        print(f"  {model}({min(20, Q - 1)};{Q}) V={V:3d}: eps_max % " + " ".join(f"{100 * x:.3f}" for x in ek)
              + f" | worst {100 * ek.max():.3f}", flush=True)
    hlb = [worst[("HLB", q)] for q in hlb_q]
    hh = [worst[("HHLB", 2 * q)] for q in hh_q]
    assert hh[0] / hh[-1] > 5 * (hlb[0] / hlb[-1]), (hlb, hh)
    for V in (40, 100, 200):
        assert worst[("HHLB", V)] < worst[("HLB", V)], V
    assert hh[-1] < 0.01 and min(hlb) > 0.01, (hlb, hh)
