"""The steady state of the stretched channel (Sec. V.C set-up: walls at
T_left = 1 and T_right = 2, g = -0.5, Kn = 0.1, Nx = 512 cells with
A = 0.9, WENO-5, f and chi with Dt = 2, CFL 0.5) against stored oracle
results, for HHLB(7;8) and for the full-range HLB(15;16).

Each stored file (tests/golden/steady_c2_*.txt, written by
make_steady_golden.py from the oracle alone) holds the step count at which
the oracle's residual max ||L[y]||_inf / ||y||_inf first fell to 1e-10 in
chunks of 1000 steps, and n, u, T after it.  The library starts from the
oracle's equilibrium (1, 0, 1), runs the same number of steps with graph
replay and must reproduce the profiles per unit mass (n / M, u, T and the
wall densities / M, M = sum_i n_i dx_i) within 1e-12 and reach the same
residual; each mass must lie within 1.5e-16 per step of the start's 1.

Why per unit mass: mass is the one mode the scheme does not damp (the walls
and the flux differences conserve it exactly in exact arithmetic).  The
rounding of a step moves it by a fraction of an ulp, with a consistent sign
near the fixed point, so over the ~4e5 steps to the steady state both
implementations drift by ~2e-11 (the oracle by 2.2e-11 for HHLB(7;8)) and
their raw densities differ by that much, uniformly.  Every damped mode
converges: the rounding difference of one step is divided by the slowest
decay rate per step (~7e-5), ~1e-12 at worst."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import check_dt, initial_states, to_oracle  # noqa: E402

import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = {"HHLB(7;8)": "steady_c2_hhlb_7_8_kn0.1.txt", "HLB(15;16)": "steady_c2_hlb_15_16_kn0.1.txt"}


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _load(path):
    head, rows = {}, []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            tag, *vals = line.split()
            if tag in ("steps", "residual", "dt", "nwall"):
                head[tag] = [float(v) for v in vals]
            else:
                rows.append([float(tag)] + [float(v) for v in vals])
    a = np.array(rows)
    return int(head["steps"][0]), head["residual"][0], head["dt"][0], np.array(head["nwall"]), a[:, 0], a[:, 1], a[:, 2]


@pytest.mark.parametrize("model", list(FILES))
def test_steady_state_against_stored_oracle(model):
    import time
    import torch
    import paper_1708_03249_amd as H
    path = os.path.join(HERE, "golden", FILES[model])
    steps, res_ref, dt_ref, nw_ref, n_ref, u_ref, T_ref = _load(path)
    quad, Q = (H.HALF_HERMITE, 8) if model.startswith("HHLB") else (H.FULL_HERMITE, 16)
    ch = H.Channel(quad=quad, Q=Q, N=Q - 1, Nx=512, adv=H.WENO5, transverse_dof=2, stretch_A=0.9,
                   Kn=0.1, g=-0.5, T_left=1.0, T_right=2.0, dt=-0.5)
    (f0, c0), = initial_states([ch])
    s = H.Solver([ch])
    try:
        d = check_dt([ch], s.dt)[0]
        assert d == dt_ref, (d, dt_ref)
        s.set_graph_steps(64)
        s.set_state(torch.from_numpy(f0.ravel()).cuda(), torch.from_numpy(c0.ravel()).cuda())
        print(f"[steady {model}] {steps} steps of dt={dt_ref:.6g}", flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[steady {model}] {1e6 * el / steps:.2f} us per step, "
              f"{ch.V * ch.Nx * steps / el:.3g} node-updates/s", flush=True)
        n, u, T = (a.cpu().numpy() for a in s.moments())
        nw, mass, bad, res = s.diagnostics(residual=True)
        assert int(bad.cpu().item()) == 0
        nw, res = nw.cpu().numpy()[0], float(res.cpu().numpy()[0])
    finally:
        s.close()
    # the mass of each solution (the start holds exactly 1): the rounding of
    # every step moves it by a fraction of an ulp with a consistent sign in
    # both implementations, and nothing damps it
    dx = O.grid(to_oracle(ch))[1]
    m, m_ref = float(np.sum(n * dx)), float(np.sum(n_ref * dx))
    en = np.abs(n / m - n_ref / m_ref).max() / (n_ref / m_ref).max()
    eu = np.abs(u - u_ref).max()          # u in units of sqrt(T_left / m)
    eT = np.abs(T - T_ref).max() / T_ref.max()
    ew = np.abs(nw / m - nw_ref / m_ref).max() / (nw_ref / m_ref).max()
    en_raw = np.abs(n - n_ref).max() / n_ref.max()
    print(f"[steady {model}] mass 1 - {1 - m:.3e} (oracle 1 - {1 - m_ref:.3e}); per unit mass: err n {en:.2e} "
          f"u {eu:.2e} T {eT:.2e} n_wall {ew:.2e} (n without the mass scaling {en_raw:.2e}); "
          f"residual {res:.3e} (oracle {res_ref:.3e})", flush=True)
    bound = 1.5e-16 * steps
    assert abs(1 - m) <= bound and abs(1 - m_ref) <= bound, (m, m_ref, bound)
    assert max(en, eu, eT, ew) <= 1e-12, (en, eu, eT, ew)
    # at 1e-10 the residual is a difference of terms 1e3 to 1e4 times larger
    # (v/dx times the populations), so its rounding is a few per cent of it
    assert res <= 1e-10 and abs(res - res_ref) <= 0.05 * res_ref, (res, res_ref)
