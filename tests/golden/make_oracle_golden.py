"""Write the oracle reference for the small-channel workload (HHLB(3;4),
Nx = 64, third-order upwind, g = -0.1, equal walls T = 1, dt = 5e-4, f and
chi, 20 000 steps from the n = 1, u = 0, T = 1 equilibrium) at
Kn = 0.01, 0.1 and 1.

Calls only the oracle.  Output: small_channel_kn<Kn>_20000.txt (the wall
densities, then f rows and chi rows, V x Nx each), repr precision.
Usage: python make_oracle_golden.py [Kn ...]"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as O  # noqa: E402

STEPS = 20000


KNS = (0.01, 0.1, 1.0)


def channel(kn):
    return O.Channel(quad=O.HALF, Q=4, N=3, Nx=64, adv=O.UPWIND3, Dt=2, L=1.0, A=0.0, Kn=kn,
                     g=-0.1, T_left=1.0, T_right=1.0, p0=1.0, dt=5e-4)


def path(kn):
    return os.path.join(HERE, f"small_channel_kn{kn:g}_{STEPS}.txt")


def write(kn):
    ch = channel(kn)
    f, chi = O.initial_state(ch)
    f2, c2, nw = O.run(ch, STEPS, f, chi)
    out = path(kn)
    with open(out, "w") as fh:
        fh.write(f"# oracle: HHLB(3;4) Nx=64 UPWIND3 Kn={kn:g} g=-0.1 T=1/1 dt=5e-4, {STEPS} steps\n")
        fh.write("# written by tests/golden/make_oracle_golden.py (calls only oracle/)\n")
        fh.write(f"# shape {f2.shape[0]} {f2.shape[1]}\n")
        fh.write("nwall " + " ".join(repr(float(x)) for x in nw) + "\n")
        for name, arr in (("f", f2), ("chi", c2)):
            for k in range(arr.shape[0]):
                fh.write(name + " " + " ".join(repr(float(x)) for x in arr[k]) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    from concurrent.futures import ThreadPoolExecutor
    kns = [float(a) for a in sys.argv[1:]] or list(KNS)
    with ThreadPoolExecutor(max_workers=len(kns)) as ex:
        list(ex.map(write, kns))
