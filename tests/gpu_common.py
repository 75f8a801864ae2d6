"""Shared helpers of the GPU parity tests: run the same seeded input through
the HIP library and the CPU oracle and compare them."""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def to_oracle(ch, dt=None):
    import paper_1708_03249_amd as H
    return O.Channel(quad=ch.quad, Q=ch.Q, N=ch.N, Nx=ch.Nx, adv=ch.adv, Dt=ch.transverse_dof,
                     L=ch.L, A=ch.stretch_A, Kn=ch.Kn, g=ch.g, T_left=ch.T_left,
                     T_right=ch.T_right, p0=ch.p0, dt=ch.dt if dt is None else dt)


def initial_states(channels, seed=0, perturb=0.0, n0=1.0, u0=0.0, T0=1.0):
    """Equilibrium initial state per channel, optionally multiplied by a seeded
    positive perturbation 1 + perturb * U[0,1) (the seeded generator holds no
    arithmetic of the method)."""
    from paper_1708_03249_amd.inputs import perturbation
    out = []
    for c, ch in enumerate(channels):
        oc = to_oracle(ch)
        f, chi = O.initial_state(oc, n0=n0, u0=u0, T0=T0)
        if perturb:
            f = f * perturbation(seed + c, f.shape, perturb)
            chi = chi * perturbation(seed + 1000 + c, f.shape, perturb)
        out.append((np.ascontiguousarray(f), np.ascontiguousarray(chi)))
    return out


def run_gpu(channels, states, nsteps, precision=0, tuning=None):
    import torch
    import paper_1708_03249_amd as H
    s = H.Solver(channels, precision=precision)
    if tuning:
        s.set_tuning(**tuning)
    f = torch.from_numpy(np.concatenate([st[0].ravel() for st in states])).cuda()
    c = torch.from_numpy(np.concatenate([st[1].ravel() for st in states])).cuda()
    s.set_state(f, c if s.has_chi else None)
    s.step(nsteps)
    fo, co = s.get_state()
    n, u, T = s.moments()
    nw, mass, bad = s.diagnostics()
    torch.cuda.synchronize()
    res = dict(f=fo.cpu().numpy(), chi=co.cpu().numpy(), n=n.cpu().numpy(), u=u.cpu().numpy(),
               T=T.cpu().numpy(), nw=nw.cpu().numpy(), mass=mass.cpu().numpy(),
               bad=int(bad.cpu().item()), offsets=s.offsets, cells=s.cells, dt=s.dt.copy())
    s.close()
    return res


def oracle_dt(ch) -> float:
    """The oracle's own time step of a channel: the given dt, or for a CFL
    request (dt < 0) min(|dt| min dx / max |p|, Kn/2) from the oracle's grid
    and nodes."""
    oc = to_oracle(ch)
    return float(ch.dt) if ch.dt > 0 else O.cfl_dt(oc, -ch.dt)


def check_dt(channels, gpu_dt, which=None):
    """The library's resolved time steps (hhlb_time_steps) against the
    oracle's own, within two ulps; returns the oracle's."""
    which = range(len(channels)) if which is None else which
    out = {}
    for c in which:
        d = oracle_dt(channels[c])
        assert abs(gpu_dt[c] - d) <= 4.5e-16 * d, (c, gpu_dt[c], d)
        out[c] = d
    return out


def run_oracle(channels, states, nsteps, gpu_dt=None, which=None, workers=8):
    """The oracle on the same inputs, with its own time step (checked
    against the library's resolved one when gpu_dt is given)."""
    which = list(range(len(channels)) if which is None else which)
    dts = check_dt(channels, gpu_dt, which) if gpu_dt is not None else \
        {c: oracle_dt(channels[c]) for c in which}

    def one(c):
        oc = to_oracle(channels[c], dt=dts[c])
        f, chi, nw = O.run(oc, nsteps, states[c][0], states[c][1])
        n, u, T = O.moments(oc, f, chi)
        return c, dict(f=f, chi=chi, nw=nw, n=n, u=u, T=T)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return dict(ex.map(one, which))


def compare(channels, gpu, ref, tol=1e-12, what=""):
    """Element-wise parity: each population within tol of the largest
    population of its cell; n and T within tol relative, u within tol of the
    thermal speed sqrt(T_left)."""
    worst = dict(f=0.0, chi=0.0, n=0.0, u=0.0, T=0.0, nw=0.0)
    for c, r in ref.items():
        ch = channels[c]
        V, Nx = ch.V, ch.Nx
        o0, o1 = gpu["offsets"][c], gpu["offsets"][c + 1]
        fg = gpu["f"][o0:o1].reshape(V, Nx)
        scale = np.abs(r["f"]).max(axis=0, keepdims=True)
        e = np.max(np.abs(fg - r["f"]) / scale)
        worst["f"] = max(worst["f"], e)
        if ch.transverse_dof:
            cg = gpu["chi"][o0:o1].reshape(V, Nx)
            sc = np.abs(r["chi"]).max(axis=0, keepdims=True)
            worst["chi"] = max(worst["chi"], np.max(np.abs(cg - r["chi"]) / sc))
        a0, a1 = gpu["cells"][c], gpu["cells"][c + 1]
        worst["n"] = max(worst["n"], np.max(np.abs(gpu["n"][a0:a1] / r["n"] - 1)))
        worst["T"] = max(worst["T"], np.max(np.abs(gpu["T"][a0:a1] / r["T"] - 1)))
        worst["u"] = max(worst["u"], np.max(np.abs(gpu["u"][a0:a1] - r["u"])) / math.sqrt(ch.T_left))
        worst["nw"] = max(worst["nw"], np.max(np.abs(gpu["nw"][c] / r["nw"] - 1)))
    bad = {k: v for k, v in worst.items() if not v <= tol}
    assert not bad, f"{what}: parity beyond {tol}: {worst}"
    return worst


def moment_errors(channels, gpu, ref):
    """Errors of the moments against the oracle: err_n = max|dn| / max n,
    err_T = max|dT| / max T, err_u = max|du| / sqrt(T_left/m), each the
    worst over the channels in ref."""
    e = dict(n=0.0, u=0.0, T=0.0)
    for c, r in ref.items():
        a0, a1 = gpu["cells"][c], gpu["cells"][c + 1]
        e["n"] = max(e["n"], np.max(np.abs(gpu["n"][a0:a1] - r["n"])) / np.max(r["n"]))
        e["T"] = max(e["T"], np.max(np.abs(gpu["T"][a0:a1] - r["T"])) / np.max(r["T"]))
        e["u"] = max(e["u"], np.max(np.abs(gpu["u"][a0:a1] - r["u"])) / math.sqrt(channels[c].T_left))
    return e


def load_golden(path):
    """(f, chi, n_wall) of a stored oracle result."""
    rows = {"f": [], "chi": []}
    nwall = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            tag, *vals = line.split()
            if tag == "nwall":
                nwall = np.array([float(v) for v in vals])
            else:
                rows[tag].append([float(v) for v in vals])
    return np.array(rows["f"]), np.array(rows["chi"]), nwall
