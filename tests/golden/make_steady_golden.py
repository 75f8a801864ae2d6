"""Write the stored oracle results of the stretched-channel steady state
(Sec. V.C: unequal walls T_left = 1, T_right = 2, g = -0.5, Kn = 0.1, Nx = 512
tanh-stretched cells with A = 0.9, WENO-5, f and chi with Dt = 2, CFL 0.5),
for HHLB(7;8) and for the full-range HLB(15;16).  Calls only the oracle.

Each model starts from the equilibrium (n, u, T) = (1, 0, 1) and advances in
chunks of 1000 RK-3 steps until the residual max over f and chi of
||L[y]||_inf / ||y||_inf (the oracle's right-hand side) is at most 1e-10;
the file stores that step count, the residual, the time step and the n, u, T
profiles and wall densities after it.  Several hours of CPU per model:

    python tests/golden/make_steady_golden.py half     # HHLB(7;8)
    python tests/golden/make_steady_golden.py full     # HLB(15;16)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

MODELS = {"half": (O.HALF, 8, "hhlb_7_8"), "full": (O.FULL, 16, "hlb_15_16")}
KN, TARGET, CHUNK = 0.1, 1e-10, 1000


def channel(which):
    quad, Q, _ = MODELS[which]
    ch = O.Channel(quad=quad, Q=Q, N=Q - 1, Nx=512, adv=O.WENO5, Dt=2, A=0.9, Kn=KN, g=-0.5,
                   T_left=1.0, T_right=2.0)
    ch.dt = O.cfl_dt(ch, 0.5)
    return ch


def residual(ch, f, chi):
    Lf, Lc, _ = O.rhs(ch, f, chi)
    return max(np.abs(Lf).max() / np.abs(f).max(), np.abs(Lc).max() / np.abs(chi).max())


def main(which):
    ch = channel(which)
    f, chi = O.initial_state(ch)
    steps, t0 = 0, time.time()
    while True:
        f, chi, nw = O.run(ch, CHUNK, f, chi)
        steps += CHUNK
        r = residual(ch, f, chi)
        if steps % 20000 == 0:
            print(f"[steady {which}] {steps} steps, residual {r:.3e}, {time.time() - t0:.0f} s", flush=True)
        if r <= TARGET:
            break
    n, u, T = O.moments(ch, f, chi)
    path = os.path.join(HERE, f"steady_c2_{MODELS[which][2]}_kn{KN:g}.txt")
    with open(path, "w") as fh:
        fh.write(f"# oracle steady state, Sec. V.C set-up: {'HHLB' if ch.quad == O.HALF else 'HLB'}"
                 f"({ch.N};{ch.Q}), Nx=512, A=0.9, WENO5, Dt=2, T_left=1, T_right=2, g=-0.5, Kn={KN:g}\n")
        fh.write("# start: equilibrium (1, 0, 1); written by tests/golden/make_steady_golden.py "
                 f"{which} (oracle only)\n")
        fh.write(f"steps {steps}\nresidual {r:.17e}\ndt {ch.dt:.17e}\n")
        fh.write(f"nwall {nw[0]:.17e} {nw[1]:.17e}\n")
        fh.write("# per cell: n u T\n")
        for i in range(ch.Nx):
            fh.write(f"{n[i]:.17e} {u[i]:.17e} {T[i]:.17e}\n")
    print(f"[steady {which}] done: {steps} steps, residual {r:.3e} -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
